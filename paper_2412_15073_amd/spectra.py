"""Vibrational spectra from the velocity autocorrelation function.

Sec. 4 of the paper reads integrator artifacts off velocity autocorrelation
spectra (resonance effects, Figs. 3-4): for water, a libration band below
1000 cm^-1, the bending peak, the stretching peaks near 3500 cm^-1; weight
beyond them comes from the time stepping (resonances) or, with jumps, from
the velocity kicks, which are white in time. This module computes
the mass-weighted spectrum

    I(nu) = sum_i m_i sum_c |sum_t w(t) v_ic(t) e^{-2 pi i nu t}|^2

from velocities sampled every step. By the Wiener-Khinchin theorem it is the
Fourier transform of the mass-weighted VACF; `vacf` gives that function in
the time domain.

Velocities are taken at every smallest time step of every scheme (the
library's velocity trace records them after each O update, i.e. at mid-step
of BAOAB and JUMP and at every inner step of the RESPA schemes), as the
paper does for its multi-time-step spectra (Sec. 4, Figs. 3-4): the Nyquist
wavenumber is 16678 cm^-1 at 1 fs, so artifacts of the outer steps (the
resonance peaks that move towards the stretch band as the outer step grows)
show up where they are. Run specs as in accuracy.py, plus "baoab_respa:n=K",
"jump_respa:n=K" (outer step K fs), and with --ewald (the same option as in
accuracy.py, or --pme for the reciprocal sum by particle-mesh Ewald)
"baoab_respa1:p=P", "jump_respa1:p=P" (1 : m : m P fs, m = 2):

    python -m paper_2412_15073_amd.spectra --n-mol 1000 --ps 4 --runs "baoab,jump,jump:eps0=0.01;rs=7"
    python -m paper_2412_15073_amd.spectra --n-mol 500 --ps 8 --pme 0.554,7,32,6,0.5 \\
        --runs "baoab,baoab_respa1:p=2,baoab_respa1:p=3,jump_respa1:p=3"
"""
import argparse
import json

import numpy as np

CM_PER_PS = 33.35640952   # 1 ps^-1 in cm^-1 (1e12 Hz / c in cm/s)

BANDS = {"libration": (0.0, 1200.0), "bend": (1200.0, 2500.0), "stretch": (2500.0, 4500.0),
         "above_stretch": (4500.0, np.inf)}


def vacf(v, mass=None, n_lags=None):
    """Mass-weighted velocity autocorrelation C(k) = < sum_i m_i v_i(t).v_i(t+k) >_t
    over all time origins, for lags 0..n_lags-1 (v: [T, N, 3])."""
    v = np.asarray(v, float)
    T = v.shape[0]
    n_lags = T if n_lags is None else n_lags
    m = np.ones(v.shape[1]) if mass is None else np.asarray(mass, float)
    x = (v * np.sqrt(m)[None, :, None]).reshape(T, -1)
    n = 1 << int(np.ceil(np.log2(2 * T)))          # zero padding: linear, not circular
    f = np.fft.rfft(x, n=n, axis=0)
    acf = np.fft.irfft((f * f.conj()).real, n=n, axis=0)[:n_lags].sum(1)
    return acf / (T - np.arange(n_lags))           # mean over the available origins


def spectrum(v, dt_ps, mass=None, window=True):
    """(wavenumbers in cm^-1, mass-weighted power spectrum normalised to unit
    sum) of velocities v [T, N, 3] sampled every dt_ps. A Hann window limits
    leakage from the finite record."""
    v = np.asarray(v, float)
    T = v.shape[0]
    m = np.ones(v.shape[1]) if mass is None else np.asarray(mass, float)
    x = v - v.mean(0, keepdims=True)
    if window:
        x = x * np.hanning(T)[:, None, None]
    f = np.fft.rfft(x, axis=0)
    p = (np.abs(f) ** 2 * m[None, :, None]).sum((1, 2))
    nu = np.fft.rfftfreq(T, d=dt_ps) * CM_PER_PS
    return nu, p / p.sum()


def band_summary(nu, p):
    """Weight and peak position of each band."""
    out = {}
    for name, (lo, hi) in BANDS.items():
        sel = (nu >= lo) & (nu < hi)
        w = float(p[sel].sum())
        out[name] = {"weight": w, "peak_cm": float(nu[sel][np.argmax(p[sel])]) if sel.any() and w > 0 else None}
    return out


def _sample(sim, step, n_calls, per_call, n_atoms, chunk):
    """Velocities [n_calls * per_call, n_atoms, 3] from the trace, fetched in
    chunks of `chunk` calls; None if the run turned unstable."""
    sim.trace_velocities(n_atoms, chunk * per_call)
    out = []
    done = 0
    while done < n_calls:
        k = min(chunk, n_calls - done)
        step(k)
        rec, _ = sim.trace()
        rec = rec[-k * per_call:]
        if not np.isfinite(rec).all():
            return None
        out.append(rec.copy())
        done += k
    return np.concatenate(out)


def main():
    from . import jumpmd, systems as S
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-mol", type=int, default=1000)
    ap.add_argument("--ps", type=float, default=4.0, help="sampled length per run")
    ap.add_argument("--equil-ps", type=float, default=5.0)
    ap.add_argument("--runs", default="baoab,jump")
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--ewald", default="", metavar="ALPHA,RC,KMAX[,W]")
    ap.add_argument("--pme", default="", metavar="ALPHA,RC,GRID,ORDER[,W]")
    a = ap.parse_args()

    ew = [float(x) for x in a.ewald.split(",")] if a.ewald else None
    pme = [float(x) for x in a.pme.split(",")] if a.pme else None
    ew = ew or (pme[:2] + [0.0] + pme[4:] if pme else None)

    def make_split(rs):
        if not ew:
            return S.water_split(r_s=rs, r_c=10.0, w=1.0, skin=0.5, n_rings=12)
        sp = S.water_split(r_s=rs, r_c=ew[1], w=ew[3] if len(ew) > 3 else 1.0, skin=0.5, alpha=ew[0],
                           n_rings=12)
        if pme:
            sp.coulomb_kind, sp.pme_grid, sp.pme_order = S.COUL_SPME, (int(pme[2]),) * 3, int(pme[3])
        else:
            sp.coulomb_kind, sp.ewald_kmax = S.COUL_EWALD, int(ew[2])
        return sp

    sysm = S.water_box(a.n_mol, seed=a.seed)
    eq = jumpmd.Sim(sysm, make_split(5.0), S.water_params(dt=0.0005, gamma=10.0, jumps=False, seed=a.seed))
    eq.step_baoab(int(round(a.equil_ps / 0.0005)))
    x, v = eq.state()
    eq.close()
    sysm.pos, sysm.vel = x, v

    dt = 0.001
    n = int(round(a.ps / dt))
    res, spectra_ = {}, {}
    for spec in a.runs.split(","):
        name, _, opts = spec.partition(":")
        kv = dict(x.split("=") for x in opts.split(";") if x)
        jumps = name.startswith("jump")
        respa = name.endswith("_respa")
        respa1 = name.endswith("_respa1")
        m = int(kv.get("n", 3)) if respa else (int(kv.get("m", 2)) if respa1 else 1)
        p_out = int(kv.get("p", 3)) if respa1 else 1
        per_call = m * p_out                         # smallest steps per call
        pa = S.water_params(dt=dt, jumps=jumps, eps0_per_kcal=float(kv.get("eps0", 0.1)), seed=a.seed + 1)
        pa.respa_inner, pa.respa_outer = m, p_out
        sim = jumpmd.Sim(sysm, make_split(float(kv.get("rs", 5.0))), pa)
        step = {"baoab": sim.step_baoab, "jump": sim.step_jump, "baoab_respa": sim.step_baoab_respa,
                "jump_respa": sim.step_jump_respa, "baoab_respa1": sim.step_baoab_respa1,
                "jump_respa1": sim.step_jump_respa1}[name]
        try:
            vs = _sample(sim, step, -(-n // per_call), per_call, sysm.n_atoms, max(1, 1000 // per_call))
            vs = vs[:n] if vs is not None else None   # the same record count in every run
        except jumpmd.MDError as e:
            vs = None
            print(f"[spectra] {spec}: {e}", flush=True)
        sim.close()
        outer_fs = dt * 1e3 * per_call
        if vs is None:
            res[spec] = {"unstable": True, "outer_step_fs": outer_fs}
            print(f"[spectra] {spec}: unstable", flush=True)
            continue
        nu, p = spectrum(vs, dt, sysm.mass)
        spectra_[spec] = p
        c = vacf(vs, sysm.mass, n_lags=200)
        hi = nu >= BANDS["above_stretch"][0]
        # weight near the harmonics of the outer-step frequency (the impulse
        # resonances of the multi-time-step schemes), +-300 cm^-1, below Nyquist
        nu_out = CM_PER_PS / (outer_fs * 1e-3)
        wins = {}
        if per_call > 1:
            for k in range(1, 5):
                c0 = k * nu_out
                if c0 + 300.0 < CM_PER_PS / (2 * dt):
                    sel = (nu > c0 - 300.0) & (nu < c0 + 300.0)
                    wins[f"{c0:.0f}"] = float(p[sel].sum())
        res[spec] = {"bands": band_summary(nu, p), "outer_step_fs": outer_fs, "outer_harmonics": wins,
                     "nyquist_cm": float(CM_PER_PS / (2 * dt)),
                     "artifact_peak_cm": float(nu[hi][np.argmax(p[hi])]),
                     "vacf_zero_crossing_fs": int(np.argmax(c < 0))}
        print(f"[spectra] {spec}: " + ", ".join(
            f"{k} {b['weight']:.4f}" + (f" @ {b['peak_cm']:.0f}" if b["peak_cm"] else "")
            for k, b in res[spec]["bands"].items()) + f", artifact peak @ {res[spec]['artifact_peak_cm']:.0f}",
            flush=True)
    if "baoab" in spectra_:
        for k, p in spectra_.items():
            if k != "baoab":
                res[k]["l1_vs_baoab"] = float(np.abs(p - spectra_["baoab"]).sum())
                print(f"[spectra] {k}: L1 vs BAOAB {res[k]['l1_vs_baoab']:.4f}, outer-step harmonics "
                      + ", ".join(f"{c} cm^-1: {w:.4f}" for c, w in res[k]["outer_harmonics"].items()), flush=True)
    print(json.dumps({"workload": f"water_{a.n_mol}mol", "ps_each": a.ps, "resolution_cm": CM_PER_PS / a.ps,
                      "electrostatics": ({"kind": "SPME", "alpha": ew[0], "r_c": ew[1], "grid": int(pme[2]),
                                          "order": int(pme[3])} if pme else
                                         {"kind": "Ewald", "alpha": ew[0], "r_c": ew[1], "kmax": int(ew[2])}
                                         if ew else {"kind": "DSF", "alpha": 0.2, "r_c": 10.0}),
                      "runs": res}), flush=True)


if __name__ == "__main__":
    main()
