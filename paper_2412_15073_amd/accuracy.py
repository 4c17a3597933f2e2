"""Sampling and dynamical accuracy of JUMP against full-range BAOAB on the GPU.

Runs the same equilibrated water box with both integrators and compares the
mean temperature, the O-O radial distribution function and the O diffusion
constant (the quantities the paper uses to validate JUMP, Sec. 4: Fig. 1
RDF/T, Fig. 2 diffusion). Prints one JSON line.

    python -m paper_2412_15073_amd.accuracy --n-mol 1000 --ps 40
"""
import argparse
import json
import time

import numpy as np

from . import analysis, jumpmd, systems as S


def run(sim, step_fn, n_steps, every, n_o, o_idx, r_max, n_bins):
    temps, frames = [], []
    counts = np.zeros(n_bins)
    nf = 0
    for _ in range(n_steps // every):
        step_fn(every)
        obs = sim.observables()
        temps.append(obs["temperature"])
        x, _ = sim.state()
        frames.append(x[o_idx].copy())
        counts += sim.rdf_counts(0, 0, r_max, n_bins)
        nf += 1
    return np.array(temps), np.array(frames), counts, nf


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-mol", type=int, default=1000)
    ap.add_argument("--ps", type=float, default=40.0, help="production length per integrator")
    ap.add_argument("--equil-ps", type=float, default=10.0)
    ap.add_argument("--eps0", type=float, default=0.1)
    ap.add_argument("--rings", type=int, default=12)
    ap.add_argument("--skin", type=float, default=0.5)
    ap.add_argument("--every", type=int, default=50, help="steps between samples")
    ap.add_argument("--precision", type=int, default=0)
    ap.add_argument("--seed", type=int, default=7)
    a = ap.parse_args()

    sysm = S.water_box(a.n_mol, seed=a.seed)
    split = S.water_split(r_s=5.0, r_c=10.0, w=1.0, skin=a.skin, n_rings=a.rings)
    L = float(sysm.box[0])
    r_max, n_bins = min(0.5 * L, 12.0), 120
    o_idx = np.where(sysm.type == 0)[0]
    n_o = len(o_idx)

    eq = jumpmd.Sim(sysm, split, S.water_params(dt=0.0005, gamma=10.0, jumps=False, seed=a.seed))
    eq.step_baoab(int(round(a.equil_ps / 0.0005)))
    x, v = eq.state()
    eq.close()
    sysm.pos, sysm.vel = x, v

    n_steps = int(round(a.ps / 0.001))
    res = {}
    for name in ("baoab", "jump"):
        pa = S.water_params(eps0_per_kcal=a.eps0, jumps=(name == "jump"), seed=a.seed + 1)
        pa.precision = a.precision
        sim = jumpmd.Sim(sysm, split, pa)
        t0 = time.perf_counter()
        T, frames, counts, nf = run(sim, sim.step_jump if name == "jump" else sim.step_baoab,
                                    n_steps, a.every, n_o, o_idx, r_max, n_bins)
        el = time.perf_counter() - t0
        r, g = analysis.rdf_from_counts(counts, n_o, n_o, L ** 3, r_max, True, nf)
        D, dD = analysis.block_diffusion(frames, a.every * 0.001, n_blocks=4)
        res[name] = dict(T=float(T.mean()), T_err=float(T.std(ddof=1) / np.sqrt(len(T))), g=g, D=D, D_err=dD,
                         seconds=el)
        sim.close()
    b, j = res["baoab"], res["jump"]
    out = {
        "workload": f"water_{a.n_mol}mol", "ps_each": a.ps, "eps0_per_kcal_mol_A": a.eps0,
        "rings": a.rings, "skin": a.skin, "precision": "fp32_mixed" if a.precision else "fp64",
        "T_baoab": b["T"], "T_jump": j["T"], "T_rel_diff": (j["T"] - b["T"]) / b["T"],
        "rdf_oo_l2": analysis.rdf_l2(b["g"], j["g"]),
        "D_baoab_A2_per_ps": b["D"], "D_baoab_err": b["D_err"],
        "D_jump_A2_per_ps": j["D"], "D_jump_err": j["D_err"], "D_rel_diff": (j["D"] - b["D"]) / b["D"],
        "targets": {"T": 0.01, "rdf_l2": 1e-2, "D": 0.05},
        "seconds": {"baoab": b["seconds"], "jump": j["seconds"]},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
