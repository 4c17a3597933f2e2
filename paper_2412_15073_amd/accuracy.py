"""Sampling and dynamical accuracy of JUMP against full-range BAOAB on the GPU.

Runs the same equilibrated water box with full-range BAOAB (FP64), JUMP
(FP64) and JUMP with FP32 pair arithmetic, and compares the mean
temperature, the mean potential energy, the O-O radial distribution function
and the O self-diffusion constant: the quantities Sec. 4 of the paper uses to
validate JUMP (temperature and RDF of water, Fig. 1; diffusion, Fig. 2).
Prints one JSON line.

    python -m paper_2412_15073_amd.accuracy --n-mol 4096 --ps 40

Run specs (--runs, comma separated): baoab, jump, baoab_respa or
jump_respa, optionally with parameters after a colon, e.g. "baoab:dt=0.5",
"jump:eps0=0.01;rs=7;fp32=1", "jump_respa:n=4" (dt in fs, the inner step of
the RESPA schemes; n inner steps per outer step, default 3; eps0 in
(kcal/mol/A)^-1; rs = split radius in A). coul= picks the
Coulomb long part's treatment in JUMP: mrz (adaptive MRZ jumps, default),
bps (BPS bounces in the C step), or none (the long part dropped: the
negative control of Fig. 1b, whose structure must differ). lj= picks the
Lennard-Jones long part's: bps (BPS bounces in the J step, default), inc
(jumps in the C step together with the Coulomb part, with its kernel) or
none (dropped).

--ewald ALPHA,RC,KMAX[,W] switches every run (and the equilibration) to
Ewald electrostatics: damped real part to RC with ALPHA, reciprocal sum over
|n| <= KMAX, switch width W (default 1 A). The schemes are then baoab and
jump (the reciprocal forces every step), baoab_respa1 and jump_respa1
(params m: middle step in inner steps, default 2; p: outer step in middle
steps, default 3). --pme ALPHA,RC,GRID,ORDER[,W] does the same with the
reciprocal sum by smooth particle-mesh Ewald on a GRID^3 mesh with B-splines
of order ORDER, e.g. the paper's water settings for 12 000 atoms (its mesh
is 60^3):

    python -m paper_2412_15073_amd.accuracy --pme 0.554,7,64,6,0.5 \
        --runs "baoab,jump,baoab_respa1:p=3,jump_respa1:p=3"
"""
import argparse
import json
import time

import numpy as np

from . import analysis, jumpmd, systems as S


def run(sim, step_fn, n_steps, every, o_idx, r_max, n_bins, t_stop):
    """Samples every `every` steps. Stops early when the kinetic temperature
    exceeds t_stop (a run that heats without bound; a transient after a change
    of potential stays well below it); returns the samples so far and the
    number of steps done."""
    temps, pes, frames = [], [], []
    counts = np.zeros(n_bins)
    for s in range(n_steps // every):
        step_fn(every)
        obs = sim.observables(pe=True)
        if not obs["temperature"] < t_stop:
            return None, (s + 1) * every, obs["temperature"]
        temps.append(obs["temperature"])
        pes.append(obs["pe_short"] + obs["pe_long"] + obs["pe_bonded"])
        x, _ = sim.state()
        frames.append(x[o_idx].copy())
        counts += sim.rdf_counts(0, 0, r_max, n_bins)
    return (np.array(temps), np.array(pes), np.array(frames), counts), n_steps, None


def block_err(x, n_blocks):
    """Standard error of the mean from n_blocks consecutive block means
    (correlated samples: the naive error understates it)."""
    x = np.asarray(x, float)
    m = len(x) // n_blocks
    b = x[: m * n_blocks].reshape(n_blocks, m).mean(1)
    return float(b.std(ddof=1) / np.sqrt(n_blocks))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-mol", type=int, default=4096)
    ap.add_argument("--ps", type=float, default=40.0, help="production length per run")
    ap.add_argument("--equil-ps", type=float, default=10.0)
    ap.add_argument("--eps0", type=float, default=0.1)
    ap.add_argument("--rings", type=int, default=12)
    ap.add_argument("--skin", type=float, default=0.5)
    ap.add_argument("--every", type=int, default=50, help="fs between samples")
    ap.add_argument("--blocks", type=int, default=4, help="blocks for the error estimates")
    ap.add_argument("--runs", default="baoab,jump,jump:fp32=1")
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--ewald", default="", metavar="ALPHA,RC,KMAX[,W]")
    ap.add_argument("--pme", default="", metavar="ALPHA,RC,GRID,ORDER[,W]")
    a = ap.parse_args()

    ew = [float(x) for x in a.ewald.split(",")] if a.ewald else None
    pme = [float(x) for x in a.pme.split(",")] if a.pme else None
    ew = ew or (pme[:2] + [0.0] + pme[4:] if pme else None)
    rc = ew[1] if ew else 10.0
    w_sw = ew[3] if ew and len(ew) > 3 else 1.0

    def make_split(rs):
        if not ew:
            return S.water_split(r_s=rs, r_c=10.0, w=1.0, skin=a.skin, n_rings=a.rings)
        sp = S.water_split(r_s=rs, r_c=rc, w=w_sw, skin=a.skin, alpha=ew[0], n_rings=a.rings)
        if pme:
            sp.coulomb_kind, sp.pme_grid, sp.pme_order = S.COUL_SPME, (int(pme[2]),) * 3, int(pme[3])
        else:
            sp.coulomb_kind, sp.ewald_kmax = S.COUL_EWALD, int(ew[2])
        return sp

    sysm = S.water_box(a.n_mol, seed=a.seed)
    split = make_split(5.0)
    L = float(sysm.box[0])
    r_max, n_bins = min(0.5 * L, 12.0), 120
    o_idx = np.where(sysm.type == 0)[0]
    n_o = len(o_idx)

    eq = jumpmd.Sim(sysm, split, S.water_params(dt=0.0005, gamma=10.0, jumps=False, seed=a.seed))
    eq.step_baoab(int(round(a.equil_ps / 0.0005)))
    x, v = eq.state()
    eq.close()
    sysm.pos, sysm.vel = x, v

    res, unstable = {}, {}
    for spec in a.runs.split(","):
        name, _, opts = spec.partition(":")
        kv = dict(x.split("=") for x in opts.split(";") if x)
        jumps = name.startswith("jump")
        respa = name.endswith("_respa")
        respa1 = name.endswith("_respa1")
        dt_fs = float(kv.get("dt", 1.0))
        n_in = int(kv.get("n", 3)) if respa else (int(kv.get("m", 2)) if respa1 else 1)
        n_out = int(kv.get("p", 3)) if respa1 else 1
        eps0 = float(kv.get("eps0", a.eps0))
        rs = float(kv.get("rs", 5.0))
        sp = make_split(rs)
        pa = S.water_params(dt=dt_fs * 1e-3, eps0_per_kcal=eps0, jumps=jumps, seed=a.seed + 1)
        pa.precision = int(kv.get("fp32", 0))
        if jumps:
            pa.jump_coul = {"mrz": S.JUMP_MRZ_ADAPTIVE, "bps": S.JUMP_BPS,
                            "none": S.JUMP_NONE}[kv.get("coul", "mrz")]
            pa.jump_lj = {"bps": S.JUMP_BPS, "none": S.JUMP_NONE, "inc": S.JUMP_IN_C}[kv.get("lj", "bps")]
        pa.respa_inner = n_in
        pa.respa_outer = n_out
        sim = jumpmd.Sim(sysm, sp, pa)
        step_fs = dt_fs * n_in * n_out                # time per call of the step function
        n_steps = int(round(a.ps / (step_fs * 1e-3)))
        every = max(1, int(round(a.every / step_fs)))
        step_fn = {"baoab": sim.step_baoab, "jump": sim.step_jump, "baoab_respa": sim.step_baoab_respa,
                   "jump_respa": sim.step_jump_respa, "baoab_respa1": sim.step_baoab_respa1,
                   "jump_respa1": sim.step_jump_respa1}[name]
        t0 = time.perf_counter()
        out_run, done, t_bad = run(sim, step_fn, n_steps, every, o_idx, r_max, n_bins, 10.0 * 300.0)
        el = time.perf_counter() - t0
        key = spec if spec not in ("jump:fp32=1",) else "jump_fp32"
        if out_run is None:
            unstable[key] = {"unstable_after_ps": done * step_fs * 1e-3, "T_K_at_stop": t_bad}
            sim.close()
            print(f"[accuracy] {spec}: unstable, T = {t_bad:.0f} K after {done * step_fs * 1e-3:.3f} ps",
                  flush=True)
            continue
        T, pe, frames, counts = out_run
        nf = len(T)
        _, g = analysis.rdf_from_counts(counts, n_o, n_o, L ** 3, r_max, True, nf)
        D, dD = analysis.block_diffusion(frames, every * step_fs * 1e-3, n_blocks=a.blocks)
        res[key] = dict(T=float(T.mean()), T_err=block_err(T, a.blocks),
                        pe=float(pe.mean()), pe_err=block_err(pe, a.blocks),
                        g=g, D=D, D_err=dD, seconds=el, ms_per_step=1e3 * el / n_steps)
        sim.close()
        print(f"[accuracy] {spec}: T {res[key]['T']:.2f} K, PE {res[key]['pe']:.1f}, D {D:.4f} +- {dD:.4f}, "
              f"{el:.1f} s", flush=True)

    ref = res.get("baoab")
    out = {"workload": f"water_{a.n_mol}mol", "ps_each": a.ps, "eps0_per_kcal_mol_A": a.eps0,
           "rings": a.rings, "skin": a.skin, "sample_every_fs": a.every,
           "electrostatics": ({"kind": "SPME", "alpha": ew[0], "r_c": rc, "grid": int(pme[2]), "order": int(pme[3]),
                               "switch": w_sw} if pme else
                              {"kind": "Ewald", "alpha": ew[0], "r_c": rc, "kmax": int(ew[2]), "switch": w_sw}
                              if ew else {"kind": "DSF", "alpha": 0.2, "r_c": 10.0, "switch": 1.0}),
           "targets": {"T_rel": 0.01, "rdf_l2": 1e-2, "D_rel": 0.05}}
    for name, r in res.items():
        row = {"T_K": r["T"], "T_err": r["T_err"], "pe_kJ_mol": r["pe"], "pe_err": r["pe_err"],
               "D_A2_per_ps": r["D"], "D_err": r["D_err"], "seconds": r["seconds"],
               "ms_per_step_with_sampling": r["ms_per_step"]}
        if ref is not None and name != "baoab":
            row["vs_baoab"] = {"T_rel": (r["T"] - ref["T"]) / ref["T"],
                               "pe_rel": (r["pe"] - ref["pe"]) / abs(ref["pe"]),
                               "rdf_l2": analysis.rdf_l2(ref["g"], r["g"]),
                               "D_rel": (r["D"] - ref["D"]) / ref["D"]}
        out[name] = row
    out.update(unstable)
    if "jump" in res and "jump_fp32" in res:
        j, f = res["jump"], res["jump_fp32"]
        out["jump_fp32"]["vs_jump_fp64"] = {"T_rel": (f["T"] - j["T"]) / j["T"],
                                            "pe_rel": (f["pe"] - j["pe"]) / abs(j["pe"]),
                                            "rdf_l2": analysis.rdf_l2(j["g"], f["g"]),
                                            "D_rel": (f["D"] - j["D"]) / j["D"]}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
