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
    a = ap.parse_args()

    seeds = [int(x) for x in a.seeds.split(",")]
    split_eq = S.water_split(r_s=5.0, r_c=10.0, w=1.0, skin=1.0, n_rings=a.rings)
    starts = {s: equilibrated(a.n_mol, s, a.equil_ps, split_eq) for s in seeds}
    L = float(starts[seeds[0]].box[0])
    r_max, n_bins = min(0.5 * L, 12.0), 120
    o_idx = np.where(starts[seeds[0]].type == 0)[0]
    n_o = len(o_idx)
    n_steps = int(round(a.ps / 1e-3))

    def measure(split, pa, scheme):
        per = []
        for s in seeds:
            p = S.Params(**{**pa.__dict__, "seed": s + 100})
            sim = jumpmd.Sim(starts[s], split, p)
            fn = sim.step_jump if scheme == "jump" else sim.step_baoab
            T, frames, counts = sample(sim, fn, n_steps, a.every, o_idx, r_max, n_bins)
            sim.close()
            _, g = analysis.rdf_from_counts(counts, n_o, n_o, L ** 3, r_max, True, len(T))
            D, dD = analysis.block_diffusion(frames, a.every * 1e-3, n_blocks=4)
            per.append({"T": float(T.mean()), "g": g, "D": D, "D_err": dD})
        pt = dict(pa.__dict__)
        pt["graph_steps"] = 20
        sim = jumpmd.Sim(starts[seeds[0]], split, S.Params(**pt))
        fn = sim.step_jump if scheme == "jump" else sim.step_baoab
        ms = timed_ms(sim, fn, a.time_steps, 40)
        sim.close()
        return per, ms

    if not a.no_reference:
        split_b = S.water_split(r_s=5.0, r_c=10.0, w=1.0, skin=1.0, n_rings=a.rings)
        per, ms = measure(split_b, S.water_params(jumps=False), "baoab")
        print(json.dumps({"point": "baoab_fp64", "ms_per_step": ms, "ns_per_day": 86.4 / ms,
                          "per_seed": [{"T": q["T"], "D": q["D"], "D_err": q["D_err"], "g": q["g"].tolist()}
                                       for q in per]}), flush=True)

    for rs in [float(x) for x in a.rs.split(",")]:
        for eps0 in [float(x) for x in a.eps0.split(",")]:
            split = S.water_split(r_s=rs, r_c=10.0, w=1.0, skin=a.skin, n_rings=a.rings)
            pa = S.water_params(eps0_per_kcal=eps0)
            pa.precision = S.FP32_MIXED
            t0 = time.perf_counter()
            per, ms = measure(split, pa, "jump")
            print(json.dumps({"point": "jump_fp32", "r_s": rs, "eps0": eps0, "ms_per_step": ms,
                              "ns_per_day": 86.4 / ms, "wall_s": time.perf_counter() - t0,
                              "per_seed": [{"T": q["T"], "D": q["D"], "D_err": q["D_err"], "g": q["g"].tolist()}
                                           for q in per]}), flush=True)


if __name__ == "__main__":
    main()
