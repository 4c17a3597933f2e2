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
the time domain. Running it compares JUMP with BAOAB on the same water box
(run specs as in accuracy.py, e.g. "jump:eps0=0.01;rs=7"):

    python -m paper_2412_15073_amd.spectra --n-mol 1000 --ps 4 --runs "baoab,jump,jump:eps0=0.01;rs=7"

The RESPA schemes (specs "baoab_respa:n=K", "jump_respa:n=K": bonded forces
every 1 fs, the rest every K fs) are sampled at their outer step, so their
spectra reach K-fold lower wavenumbers (Nyquist 16678/K cm^-1, the stretch
band aliased from K = 5 on); each is compared with the 1 fs BAOAB run
subsampled at the same interval, so that the aliasing is the same on both
sides and the difference is that of the integrators (the resonances of
Sec. 4, Figs. 3-4):

    python -m paper_2412_15073_amd.spectra --n-mol 1000 --ps 8 --runs "baoab,baoab_respa:n=3,jump_respa:n=3"
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


def main():
    from . import jumpmd, systems as S
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-mol", type=int, default=1000)
    ap.add_argument("--ps", type=float, default=4.0, help="sampled length per run")
    ap.add_argument("--equil-ps", type=float, default=5.0)
    ap.add_argument("--runs", default="baoab,jump")
    ap.add_argument("--seed", type=int, default=7)
    a = ap.parse_args()

    sysm = S.water_box(a.n_mol, seed=a.seed)
    split = S.water_split(r_s=5.0, r_c=10.0, w=1.0, skin=0.5, n_rings=12)
    eq = jumpmd.Sim(sysm, split, S.water_params(dt=0.0005, gamma=10.0, jumps=False, seed=a.seed))
    eq.step_baoab(int(round(a.equil_ps / 0.0005)))
    x, v = eq.state()
    eq.close()
    sysm.pos, sysm.vel = x, v

    dt = 0.001
    n = int(round(a.ps / dt))
    res, spectra_ = {}, {}
    v_baoab = None
    for spec in a.runs.split(","):
        name, _, opts = spec.partition(":")
        kv = dict(x.split("=") for x in opts.split(";") if x)
        jumps = name.startswith("jump")
        respa = name.endswith("_respa")
        k_out = int(kv.get("n", 3)) if respa else 1
        sp = S.water_split(r_s=float(kv.get("rs", 5.0)), r_c=10.0, w=1.0, skin=0.5, n_rings=12)
        pa = S.water_params(dt=dt, jumps=jumps, eps0_per_kcal=float(kv.get("eps0", 0.1)), seed=a.seed + 1)
        pa.respa_inner = k_out
        sim = jumpmd.Sim(sysm, sp, pa)
        step = {"baoab": sim.step_baoab, "jump": sim.step_jump, "baoab_respa": sim.step_baoab_respa,
                "jump_respa": sim.step_jump_respa}[name]
        n_s = n // k_out
        vs = np.empty((n_s, sysm.n_atoms, 3))
        for t in range(n_s):
            step(1)
            vs[t] = sim.state()[1]
        sim.close()
        if name == "baoab":
            v_baoab = vs
        nu, p = spectrum(vs, dt * k_out, sysm.mass)
        spectra_[spec] = (k_out, p)
        c = vacf(vs, sysm.mass, n_lags=max(2, 200 // k_out))
        res[spec] = {"bands": band_summary(nu, p), "sample_fs": k_out,
                     "nyquist_cm": float(CM_PER_PS / (2 * dt * k_out)),
                     "vacf_zero_crossing_fs": int(np.argmax(c < 0)) * k_out}
        print(f"[spectra] {spec}: " + ", ".join(
            f"{k} {b['weight']:.3f}" + (f" @ {b['peak_cm']:.0f}" if b["peak_cm"] else "")
            for k, b in res[spec]["bands"].items()), flush=True)
    if v_baoab is not None:
        for k, (k_out, p) in spectra_.items():
            if k == "baoab":
                continue
            # the reference at the same sampling interval (same aliasing)
            nu_r, p_r = spectrum(v_baoab[k_out - 1::k_out], dt * k_out, sysm.mass)
            m = min(len(p), len(p_r))
            res[k]["l1_vs_baoab"] = float(np.abs(p[:m] - p_r[:m]).sum())
            if k_out > 1:
                res[k]["baoab_subsampled_bands"] = band_summary(nu_r, p_r)
    print(json.dumps({"workload": f"water_{a.n_mol}mol", "ps_each": a.ps, "resolution_cm": CM_PER_PS / a.ps,
                      "runs": res}), flush=True)


if __name__ == "__main__":
    main()
