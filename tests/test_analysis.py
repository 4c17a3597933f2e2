"""Host-side analysis (RDF normalisation, Einstein diffusion, VACF spectra)
against closed forms and brute force."""
import numpy as np

from paper_2412_15073_amd import analysis, spectra


def test_rdf_of_uniform_points_is_one():
    """Ideal gas: uniformly placed points in a periodic box have g(r) = 1.
    Histogram by brute force over minimum-image pairs, normalised by
    rdf_from_counts."""
    rng = np.random.default_rng(1)
    L, n, frames, r_max, nb = 10.0, 200, 20, 4.0, 8
    counts = np.zeros(nb)
    for _ in range(frames):
        x = rng.uniform(0, L, (n, 3))
        d = x[:, None, :] - x[None, :, :]
        d -= L * np.rint(d / L)
        r = np.sqrt((d * d).sum(-1))[np.triu_indices(n, 1)]
        counts += np.histogram(r, bins=nb, range=(0.0, r_max))[0]
    _, g = analysis.rdf_from_counts(counts, n, n, L ** 3, r_max, True, frames)
    assert np.all(np.abs(g[2:] - 1.0) < 0.06), g        # inner bins hold few pairs
    assert abs(g[1:].mean() - 1.0) < 0.03


def test_einstein_diffusion_of_a_random_walk():
    """Brownian walk with D = 0.3: each coordinate steps N(0, 2 D dt), so the
    MSD is 6 D t and the fit returns D."""
    rng = np.random.default_rng(2)
    D, dt, T, n = 0.3, 0.05, 400, 500
    steps = rng.normal(0.0, np.sqrt(2 * D * dt), (T, n, 3))
    frames = np.cumsum(steps, axis=0)
    m = analysis.msd(frames)
    assert abs(m[1] - 6 * D * dt) < 0.05 * 6 * D * dt
    est, err = analysis.block_diffusion(frames, dt, n_blocks=4)
    assert abs(est - D) < 0.05 * D and err < 0.05 * D


def test_vacf_matches_brute_force():
    rng = np.random.default_rng(3)
    T, n = 37, 4
    v = rng.standard_normal((T, n, 3))
    m = rng.uniform(1.0, 16.0, n)
    c = spectra.vacf(v, m, n_lags=T)
    for k in range(T):
        ref = np.mean([(m[:, None] * v[t] * v[t + k]).sum() for t in range(T - k)])
        assert abs(c[k] - ref) < 1e-10 * abs(ref) + 1e-12


def test_spectrum_peaks_at_the_oscillation_wavenumbers():
    """Two atoms oscillating at 1650 and 3600 cm^-1 (1 fs sampling, 4 ps):
    the spectrum peaks at those wavenumbers (within one bin of 8.3 cm^-1),
    splits its weight by the mass-weighted energies, and has none beyond the
    stretch band."""
    dt, T = 0.001, 4000
    t = np.arange(T) * dt
    nu1, nu2 = 1650.0, 3600.0
    v = np.zeros((T, 2, 3))
    v[:, 0, 0] = np.cos(2 * np.pi * nu1 / spectra.CM_PER_PS * t)
    v[:, 1, 1] = 2.0 * np.sin(2 * np.pi * nu2 / spectra.CM_PER_PS * t + 0.3)
    m = np.array([16.0, 1.0])
    nu, p = spectra.spectrum(v, dt, m)
    res = spectra.CM_PER_PS / (T * dt)
    b = spectra.band_summary(nu, p)
    assert abs(b["bend"]["peak_cm"] - nu1) <= res and abs(b["stretch"]["peak_cm"] - nu2) <= res
    # weights m a^2 / 2: 16 * 1 vs 1 * 4
    assert abs(b["bend"]["weight"] - 0.8) < 0.01 and abs(b["stretch"]["weight"] - 0.2) < 0.01
    assert b["above_stretch"]["weight"] < 1e-6


def test_frontier_summary_names_the_fastest_point_within_targets(tmp_path, capsys):
    """The frontier table: errors against the 1 fs reference, targets
    (T 1 %, RDF L2 1e-2, D 5 %) and the fastest JUMP point meeting all."""
    import json
    from paper_2412_15073_amd import frontier
    g = [1.0] * 10

    def pt(point, ms, T, D, dg=0.0, **kw):
        seeds = [{"T": T, "D": D, "D_err": 0.001, "g": [x + dg for x in g]} for _ in range(2)]
        return json.dumps({"point": point, "ms_per_step": ms, "ns_per_day": 86.4 * kw.get("dt_fs", 1.0) / ms,
                           "per_seed": seeds, **kw})
    lines = [pt("baoab_fp64", 0.1, 300.0, 0.25, dt_fs=1.0),
             pt("jump_fp32", 0.08, 301.0, 0.24, r_s=7.0, eps0=0.01, dt_fs=1.0),     # meets all, fastest
             pt("jump_fp32", 0.05, 300.0, 0.10, r_s=5.0, eps0=0.1, dt_fs=1.0),      # D off by 60 %
             pt("jump_fp32", 0.09, 300.5, 0.25, r_s=9.0, eps0=0.01, dt_fs=1.0),     # meets all, slower
             pt("jump_fp32", 0.06, 300.0, 0.25, dg=0.05, r_s=6.0, eps0=0.03, dt_fs=1.0)]   # RDF off
    f = tmp_path / "log"
    f.write_text("noise\n" + "\n".join(lines) + "\n")
    frontier.summarize([str(f)])
    out = capsys.readouterr().out
    assert "fastest JUMP point meeting all targets: JUMP FP32 r_s 7 eps0 0.01" in out
    assert "1080.0 ns/day (1.25x" in out
