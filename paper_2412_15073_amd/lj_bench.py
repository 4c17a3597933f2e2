"""Timing of the Lennard-Jones workload on the GPU: 864 atoms on an fcc
lattice (reduced density 0.8442, kT 0.722, dt 0.005, gamma 1), JUMP as
B J A O A J B with BPS jumps on the LJ long part between r_s = 3 sigma and
r_c = 5 sigma (Sec. 3.2, Alg. 5), against BAOAB with the full-range force.
After an untimed BAOAB equilibration, each integrator runs `--runs` timed
blocks of `--steps` steps (replayed as HIP graphs); the median block gives
steps/s and tau/day. Prints one JSON line.

    python -m paper_2412_15073_amd.lj_bench
"""
import argparse
import json
import time

import numpy as np

from . import jumpmd, systems as S


def _time_blocks(sim, step_fn, steps, runs):
    out = []
    for _ in range(runs):
        sim.sync()
        t0 = time.perf_counter()
        step_fn(steps)
        sim.sync()
        out.append(time.perf_counter() - t0)
    return float(np.median(out)), out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--equil", type=int, default=10000, help="untimed BAOAB steps")
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--runs", type=int, default=5)
    ap.add_argument("--rings", type=int, default=1)
    ap.add_argument("--graph-steps", type=int, default=20)
    a = ap.parse_args()

    sysm = S.lj_fcc(6, seed=1)
    sp_jump = S.lj_split(skin=0.3, n_rings=a.rings,
                         ring_width=0.0 if a.rings == 1 else (5.3 - 2.2) / a.rings)
    pa_eq = S.lj_params(jumps=False)
    eq = jumpmd.Sim(sysm, sp_jump, pa_eq)
    eq.step_baoab(a.equil)
    x, v = eq.state()
    eq.close()
    sysm.pos, sysm.vel = x, v

    res = {}
    for name, jumps in (("jump", True), ("baoab_full", False)):
        pa = S.lj_params(seed=2, jumps=jumps)
        pa.graph_steps = a.graph_steps
        sim = jumpmd.Sim(sysm, sp_jump, pa)
        step_fn = sim.step_jump if jumps else sim.step_baoab
        step_fn(2 * a.graph_steps)                      # warm-up: graphs captured, rows built
        p0 = sim.proposals_total() if jumps else 0
        med, all_s = _time_blocks(sim, step_fn, a.steps, a.runs)
        obs = sim.observables()
        props = (sim.proposals_total() - p0) / (a.steps * a.runs) if jumps else 0.0
        sim.close()
        sps = a.steps / med
        res[name] = {"ms_per_step": 1e3 * med / a.steps, "steps_per_s": sps,
                     "tau_per_day": sps * pa.dt * 86400.0, "T": obs["temperature"],
                     "proposals_per_step": props, "block_seconds": all_s}
        print(f"[lj_bench] {name}: {res[name]['ms_per_step']:.4f} ms/step, "
              f"{res[name]['tau_per_day']:.0f} tau/day, T = {obs['temperature']:.3f}", flush=True)
    res["jump_speedup_vs_baoab"] = res["jump"]["steps_per_s"] / res["baoab_full"]["steps_per_s"]
    print(json.dumps({"workload": "lj_fcc_864", "rings": a.rings, "steps": a.steps, "runs": a.runs,
                      "graph_steps": a.graph_steps, **res}), flush=True)


if __name__ == "__main__":
    main()
