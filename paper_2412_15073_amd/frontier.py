"""Speed against accuracy of JUMP over its tuning parameters (Sec. 4,
"Tuning of parameters": the split radius and eps0 trade speed against the
diffusion constant) on the 4096-water box.

For every (r_s, eps0) point of the grid, JUMP (FP32-mixed pair arithmetic,
the benchmark's precision; LJ BPS + Coulomb adaptive MRZ, shell r_s - 1 ...
r_c = 10 A) runs from the same BAOAB-equilibrated starts as the FP64 BAOAB
reference (full-range forces, 1 fs); each start gives the mean temperature,
the O-O radial distribution function and the O self-diffusion constant, and
the point's speed is timed separately (HIP-graph replays, no sampling). The
matched-accuracy targets are those of the comparison: T within 1 %, RDF
within 1e-2 (L2 over bins), D within 5 % of BAOAB. Prints one JSON line per
point (and per reference), so that a long grid can be run in pieces.

    python -m paper_2412_15073_amd.frontier --rs 5,7,9 --eps0 0.003,0.01,0.03,0.1 --seeds 7,8

With --pme ALPHA,RC,GRID,ORDER,W the electrostatics are Ewald (damped real
part to RC, particle-mesh reciprocal sum every step in JUMP's acceleration
and BAOAB's kicks), e.g. the paper's settings for its 12 000-atom water:
--pme 0.554,7,64,6,0.5 --rs 5,6.

The reference runs (FP64 BAOAB at 1 fs, and at 0.5 fs as a check of the
1 fs reference's own time-step error) are printed first. `--summarize`
reads such JSON lines back (from any number of logs) and prints the table
of every point against the 1 fs reference, with the targets met or not (and
the temperature against the 0.5 fs reference: BAOAB's kinetic temperature at
1 fs reads low for flexible water):

    python -m paper_2412_15073_amd.frontier --summarize log1 log2 ...
"""
import argparse
import json
import time

import numpy as np

from . import analysis, jumpmd, systems as S


def equilibrated(n_mol, seed, equil_ps, split):
    sysm = S.water_box(n_mol, seed=seed)
    eq = jumpmd.Sim(sysm, split, S.water_params(dt=0.0005, gamma=10.0, jumps=False, seed=seed))
    eq.step_baoab(int(round(equil_ps / 0.0005)))
    x, v = eq.state()
    eq.close()
    sysm.pos, sysm.vel = x, v
    return sysm


def sample(sim, step_fn, n_steps, every, o_idx, r_max, n_bins):
    temps, frames = [], []
    counts = np.zeros(n_bins)
    for _ in range(n_steps // every):
        step_fn(every)
        temps.append(sim.observables()["temperature"])
        x, _ = sim.state()
        frames.append(x[o_idx].copy())
        counts += sim.rdf_counts(0, 0, r_max, n_bins)
    return np.array(temps), np.array(frames), counts


def timed_ms(sim, step_fn, steps, warmup):
    import torch
    step_fn(warmup)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_fn(steps)
    sim.sync()
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0) / steps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-mol", type=int, default=4096)
    ap.add_argument("--rs", default="5,6,7,8,9", help="split radii (A); switch width 1 A below each")
    ap.add_argument("--eps0", default="0.003,0.01,0.03,0.1", help="adaptive eps0 values, (kcal/mol/A)^-1")
    ap.add_argument("--seeds", default="7,8", help="independent starts (lattice, velocities, streams)")
    ap.add_argument("--ps", type=float, default=20.0, help="production per start")
    ap.add_argument("--equil-ps", type=float, default=10.0)
    ap.add_argument("--every", type=int, default=50, help="fs between samples")
    ap.add_argument("--time-steps", type=int, default=300)
    ap.add_argument("--skin", type=float, default=0.5)
    ap.add_argument("--rings", type=int, default=12)
    ap.add_argument("--no-reference", action="store_true")
    ap.add_argument("--ref-dt", default="1.0,0.5", help="time steps (fs) of the FP64 BAOAB references")
    ap.add_argument("--summarize", nargs="+", metavar="LOG", help="summarise logs of earlier runs and exit")
    ap.add_argument("--lj", default="bps", choices=("bps", "inc"),
                    help="LJ long part: BPS bounces in the J step, or jumps in the C step with the Coulomb part")
    ap.add_argument("--pme", default="", metavar="ALPHA,RC,GRID,ORDER,W",
                    help="Ewald electrostatics (particle-mesh reciprocal sum) instead of DSF to 10 A")
    a = ap.parse_args()
    if a.summarize:
        summarize(a.summarize)
        return

    seeds = [int(x) for x in a.seeds.split(",")]
    pme = [float(x) for x in a.pme.split(",")] if a.pme else None

    def make_split(rs, skin):
        if not pme:
            return S.water_split(r_s=rs, r_c=10.0, w=1.0, skin=skin, n_rings=a.rings)
        sp = S.water_split(r_s=rs, r_c=pme[1], w=pme[4], skin=skin, alpha=pme[0], n_rings=a.rings)
        sp.coulomb_kind, sp.pme_grid, sp.pme_order = S.COUL_SPME, (int(pme[2]),) * 3, int(pme[3])
        return sp

    split_eq = make_split(5.0, 1.0)
    starts = {s: equilibrated(a.n_mol, s, a.equil_ps, split_eq) for s in seeds}
    L = float(starts[seeds[0]].box[0])
    r_max, n_bins = min(0.5 * L, 12.0), 120
    o_idx = np.where(starts[seeds[0]].type == 0)[0]
    n_o = len(o_idx)
    n_steps = int(round(a.ps / 1e-3))

    def measure(split, pa, scheme):
        per = []
        step_fs = pa.dt * 1e3
        n_run = int(round(a.ps / (step_fs * 1e-3)))
        every = max(1, int(round(a.every / step_fs)))
        for s in seeds:
            p = S.Params(**{**pa.__dict__, "seed": s + 100})
            sim = jumpmd.Sim(starts[s], split, p)
            fn = sim.step_jump if scheme == "jump" else sim.step_baoab
            T, frames, counts = sample(sim, fn, n_run, every, o_idx, r_max, n_bins)
            sim.close()
            _, g = analysis.rdf_from_counts(counts, n_o, n_o, L ** 3, r_max, True, len(T))
            D, dD = analysis.block_diffusion(frames, every * step_fs * 1e-3, n_blocks=4)
            per.append({"T": float(T.mean()), "g": g, "D": D, "D_err": dD})
        pt = dict(pa.__dict__)
        pt["graph_steps"] = 20
        sim = jumpmd.Sim(starts[seeds[0]], split, S.Params(**pt))
        fn = sim.step_jump if scheme == "jump" else sim.step_baoab
        ms = timed_ms(sim, fn, a.time_steps, 40)
        sim.close()
        return per, ms

    if not a.no_reference:
        split_b = make_split(5.0, 1.0)
        for dt_fs in [float(x) for x in a.ref_dt.split(",")]:
            per, ms = measure(split_b, S.water_params(dt=dt_fs * 1e-3, jumps=False), "baoab")
            print(json.dumps({"point": "baoab_fp64", "dt_fs": dt_fs, "ms_per_step": ms, "pme": a.pme or None,
                              "ns_per_day": 86.4 * dt_fs / ms, "r_max": r_max,
                              "per_seed": [{"T": q["T"], "D": q["D"], "D_err": q["D_err"], "g": q["g"].tolist()}
                                           for q in per]}), flush=True)

    for rs in [float(x) for x in a.rs.split(",") if x]:    # --rs "": the references only
        for eps0 in [float(x) for x in a.eps0.split(",") if x]:
            split = make_split(rs, a.skin)
            pa = S.water_params(eps0_per_kcal=eps0)
            pa.precision = S.FP32_MIXED
            if a.lj == "inc":
                pa.jump_lj = S.JUMP_IN_C
            t0 = time.perf_counter()
            per, ms = measure(split, pa, "jump")
            print(json.dumps({"point": "jump_fp32", "r_s": rs, "eps0": eps0, "dt_fs": 1.0, "ms_per_step": ms,
                              "pme": a.pme or None, "lj": a.lj,
                              "ns_per_day": 86.4 / ms, "wall_s": time.perf_counter() - t0,
                              "per_seed": [{"T": q["T"], "D": q["D"], "D_err": q["D_err"], "g": q["g"].tolist()}
                                           for q in per]}), flush=True)


TARGETS = {"T_rel": 0.01, "rdf_l2": 1e-2, "D_rel": 0.05}


def _combine(point):
    """Mean over seeds: T, g, D, and the standard error of D (block errors
    of each seed combined with the spread between seeds)."""
    per = point["per_seed"]
    T = float(np.mean([q["T"] for q in per]))
    g = np.mean([q["g"] for q in per], axis=0)
    Ds = np.array([q["D"] for q in per])
    e_block = np.sqrt(np.sum([q["D_err"] ** 2 for q in per])) / len(per)
    e_seed = Ds.std(ddof=1) / np.sqrt(len(Ds)) if len(Ds) > 1 else 0.0
    return T, g, float(Ds.mean()), float(max(e_block, e_seed))


def summarize(logs):
    pts = []
    for f in logs:
        with open(f) as fh:
            for line in fh:
                line = line.strip()
                if line.startswith("{") and '"point"' in line:
                    pts.append(json.loads(line))
    kinds = sorted({str(p.get("pme")) for p in pts})
    if len(kinds) > 1:   # one table per electrostatics
        for k in kinds:
            print(f"electrostatics: {'DSF, r_c 10 A' if k == 'None' else 'Ewald ' + k}")
            _table([p for p in pts if str(p.get("pme")) == k])
        return
    _table(pts)


def _table(pts):
    refs = {p["dt_fs"]: p for p in pts if p["point"] == "baoab_fp64"}
    ref = refs.get(1.0)
    assert ref is not None, "no 1 fs BAOAB reference in the logs"
    T0, g0, D0, e0 = _combine(ref)
    T05 = _combine(refs[0.5])[0] if 0.5 in refs else None
    rows = []
    for p in pts:
        T, g, D, e = _combine(p)
        dT = (T - T0) / T0
        l2 = float(np.sqrt(np.mean((g - g0) ** 2)))
        dD = (D - D0) / D0
        ok = abs(dT) <= TARGETS["T_rel"] and l2 <= TARGETS["rdf_l2"] and abs(dD) <= TARGETS["D_rel"]
        name = (f"BAOAB FP64 {p['dt_fs']:g} fs" if p["point"] == "baoab_fp64"
                else f"JUMP FP32 r_s {p['r_s']:g} eps0 {p['eps0']:g}" + (" LJ in C" if p.get("lj") == "inc" else ""))
        dT05 = (T - T05) / T05 if T05 else float("nan")
        rows.append((name, p["ms_per_step"], p["ns_per_day"], T, dT, l2, D, e, dD, ok, dT05))
    print(f"{'run':34s} {'ms/step':>8s} {'ns/day':>8s} {'T (K)':>8s} {'dT':>7s} {'dT.5fs':>7s} {'RDF L2':>7s} "
          f"{'D':>7s} {'+-':>6s} {'dD':>7s}  all targets")
    for r in rows:
        print(f"{r[0]:34s} {r[1]:8.4f} {r[2]:8.1f} {r[3]:8.2f} {100 * r[4]:6.2f}% {100 * r[10]:6.2f}% {r[5]:7.4f} "
              f"{r[6]:7.4f} {r[7]:6.4f} {100 * r[8]:6.1f}%  {'yes' if r[9] else 'no'}")
    best = [r for r in rows if r[9] and r[0].startswith("JUMP")]
    if best:
        b = max(best, key=lambda r: r[2])
        print(f"fastest JUMP point meeting all targets: {b[0]}, {b[2]:.1f} ns/day "
              f"({b[2] / ref['ns_per_day']:.2f}x the 1 fs BAOAB reference)")
    else:
        print("no JUMP point meets all targets")


if __name__ == "__main__":
    main()
