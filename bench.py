#!/usr/bin/env python
"""Throughput of the JUMP hot path on one MI355X, with full-range BAOAB beside it.

Workload (default): flexible 3-site water, 4096 molecules (12288 atoms) in a
49.7 A box at 300 K, FP64; pair potentials split at r_s = 5 A (switch 1 A),
long part out to r_c = 10 A handled by jumps (LJ: BPS, Coulomb: adaptive MRZ,
eps0 = 0.1 (kcal/mol/A)^-1), dt = 1 fs, gamma = 1/ps. The comparator
integrates the same system with BAOAB and full-range (r < r_c) forces.
Inputs are synthetic (lattice start, then an untimed BAOAB equilibration);
everything timed is resident in HBM.

Timed region: K steps replayed as HIP graphs of --graph-steps steps (plain
launches with --graph-steps 0). Per-kernel durations for the roofline come
from a second, profiled run of plain launches in the same process (HIP events
on the library's stream).

Prints ONE JSON line. --gpus N > 1 exits: the benchmark runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6      # MI355X dense FP64 vector: 256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0

# Algorithmic work units, counted from the formulas (one flop per add, mul,
# fma, division, square root or transcendental call):
#  a short-range pair term: chi * (LJ + DSF) and its gradient, 78 flops;
#  a full-range pair term (BAOAB comparator): LJ + DSF and gradient, 60 flops;
#  a jump proposal: long-range pair gradient (1 - chi) U, rate at the
#  proposal time, clock and acceptance, 93 flops.
FLOP_PER_SHORT_PAIR = 78
FLOP_PER_FULL_PAIR = 60
FLOP_PER_PROPOSAL = 93
BYTES_PER_ATOM_LOCAL = 7 * 32   # x (read+write), v (read+write), f_nb, f_b, x_ref reads
# HBM bytes per launch of the chain kernel from FETCH_SIZE / WRITE_SIZE counters
# scaled by a 256 MiB copy (profiles/k_chain_water4096_fp64.md), valid while the
# sha256 of the chain kernel's sources (md_chain.hip, then md_device.h) starts
# with the given prefix, default workload only.
CHAIN_TRAFFIC = {"sha256": "35aa22ab282dcad4", "bytes": 37496513,
                 "workload": ("fp64", 4096, 12, 0.5, 0.1, 0, False, 10.0)}
KERNELS = {0: "k_local (B/A/O updates)", 1: "k_force (pairs, with bonded when fused)", 2: "k_bonded (separate)", 3: "row rebuild",
           4: "k_chain (J/C jump chains)"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--equil", type=int, default=4000, help="untimed BAOAB steps at 0.5 fs, gamma 10/ps")
    ap.add_argument("--n-mol", type=int, default=4096)
    ap.add_argument("--eps0", type=float, default=0.1, help="adaptive eps0 in (kcal/mol/A)^-1")
    ap.add_argument("--rings", type=int, default=12)
    ap.add_argument("--skin", type=float, default=0.5)
    ap.add_argument("--baoab-skin", type=float, default=1.0,
                    help="list skin of the BAOAB comparator (its fastest; JUMP's fastest is 0.5)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-baoab", action="store_true")
    ap.add_argument("--chain-lanes", type=int, default=0, help="lanes per atom in the jump chains (0 = auto)")
    ap.add_argument("--graph-steps", type=int, default=20, help="steps per replayed HIP graph (0 = plain launches)")
    ap.add_argument("--profile-steps", type=int, default=200, help="plain-launch steps timed per kernel")
    ap.add_argument("--precision", choices=("fp64", "fp32"), default="fp64",
                    help="pair arithmetic of forces and jump rates (fp32: mixed, FP64 state)")
    ap.add_argument("--replicas", type=int, default=0,
                    help="batched ensemble: R water replicas of U{216..2048} molecules (seed 1) in one context")
    ap.add_argument("--respa", action="store_true",
                    help="JUMP-RESPA vs BAOAB-RESPA: bonded forces every 1 fs, the rest every --respa-inner fs")
    ap.add_argument("--respa-inner", type=int, default=3)
    ap.add_argument("--rc", type=float, default=10.0, help="outer cutoff of the jumped shell (A)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (HBM counter calibration) and exit")
    return ap.parse_args()


def calibrate_copy(mib):
    import torch
    n = mib * (1 << 20) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 5}), flush=True)


def timed(sim, fn, steps, warmup):
    import torch
    fn(warmup)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fn(steps)
    sim.sync()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def kernel_profile(sim, fn, steps):
    """Per-kernel totals (ms) and launch counts over `steps` plain-launch steps."""
    import torch
    sim.sync()
    torch.cuda.synchronize()
    sim.profile(True)
    fn(steps)
    sim.sync()
    prof = {k: sim.profile_read(k) for k in KERNELS}
    sim.profile(False)
    return prof


def ns_per_day(dt_ps, steps, seconds):
    return dt_ps * 1e-3 * (steps / seconds) * 86400.0


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on exactly one GPU; --gpus must be 1",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench needs a GPU"
    if a.calibrate_copy:
        calibrate_copy(a.calibrate_copy)
        return
    import ctypes as C
    from paper_2412_15073_amd import jumpmd, systems as S

    prec = 1 if a.precision == "fp32" else 0
    # replicas below 267 molecules (box < 20 A) cannot hold r_c = 10 A under the
    # minimum-image convention: the ensemble's sizes are drawn from U{270..2048}
    n_min = 270 if a.rc >= 10.0 else 216
    if a.replicas:
        sysm = S.water_replicas(a.replicas, n_min=n_min, seed=1)
        n_atoms = int(sysm.offsets[-1])
        desc = f"{a.replicas} water replicas, {n_atoms // 3} molecules ({n_atoms} atoms) in total"
    else:
        sysm = S.water_box(a.n_mol, seed=1)
        n_atoms = sysm.n_atoms
        desc = f"water {a.n_mol} molecules ({n_atoms} atoms), box {sysm.box[0]:.2f} A"
    split = S.water_split(r_s=5.0, r_c=a.rc, w=1.0, skin=a.skin, n_rings=a.rings)
    n_sys = max(1, a.replicas)
    if a.respa:
        a.graph_steps = 0   # graph replay covers the single-step schemes only
    print(f"[bench] {desc}", flush=True)

    def set_state(sy, x, v):
        if a.replicas:
            for r, s_r in enumerate(sy.systems):
                lo, hi = sy.offsets[r], sy.offsets[r + 1]
                s_r.pos, s_r.vel = x[lo:hi], v[lo:hi]
        else:
            sy.pos, sy.vel = x, v

    def fresh_system():
        return S.water_replicas(a.replicas, n_min=n_min, seed=1) if a.replicas else S.water_box(a.n_mol, seed=1)

    # untimed equilibration from the lattice: BAOAB, full forces, 0.5 fs, gamma 10/ps
    eq = jumpmd.Sim(sysm, split, S.water_params(dt=0.0005, gamma=10.0, jumps=False))
    t = time.perf_counter()
    eq.step_baoab(a.equil)
    obs = eq.observables()
    x, v = eq.state()
    eq.close()
    print(f"[bench] equilibrated {a.equil} steps in {time.perf_counter() - t:.1f} s, T = {obs['temperature']:.1f} K",
          flush=True)
    set_state(sysm, x, v)

    def params(jumps, graph):
        p = S.water_params(eps0_per_kcal=a.eps0, jumps=jumps)
        p.chain_lanes = a.chain_lanes
        p.graph_steps = graph
        p.precision = prec
        if a.respa:
            p.respa_inner = a.respa_inner
        return p

    def jstep(sim):
        return sim.step_jump_respa if a.respa else sim.step_jump

    def bstep(sim):
        return sim.step_baoab_respa if a.respa else sim.step_baoab

    step_ps = 1e-3 * (a.respa_inner if a.respa else 1)   # simulated time per call step
    name_j, name_b = ("JUMP-RESPA", "BAOAB-RESPA") if a.respa else ("JUMP", "BAOAB-full")

    # JUMP (C' J' A O A J' C', or its RESPA form): timed run
    pj = params(True, a.graph_steps)
    js = jumpmd.Sim(sysm, split, pj)
    p0 = js.proposals_total()
    dt_j = timed(js, jstep(js), a.steps, a.warmup)
    props = (js.proposals_total() - p0) / (a.steps + a.warmup)
    obs_j = js.observables()
    pl, pt = C.c_int64(0), C.c_int64(0)
    jumpmd.load().md_counters(js._h, C.byref(pl), C.byref(pt))
    pairs_short = pl.value
    xj, vj = js.state()
    js.close()
    ms_j = 1e3 * dt_j / a.steps
    ns_day_j = n_sys * ns_per_day(step_ps, a.steps, dt_j)
    print(f"[bench] {name_j} {ms_j:.4f} ms/step, {ns_day_j:.1f} ns/day, T = {obs_j['temperature']:.1f} K, "
          f"{props:.0f} proposals/step, {pairs_short} short pairs", flush=True)

    # JUMP per-kernel profile: plain launches from the timed run's final state
    s2 = fresh_system()
    set_state(s2, xj, vj)
    jp = jumpmd.Sim(s2, split, params(True, 0))
    jstep(jp)(a.warmup)
    q0 = jp.proposals_total()
    prof_j = kernel_profile(jp, jstep(jp), a.profile_steps)
    props_prof = (jp.proposals_total() - q0) / a.profile_steps
    jp.close()

    # BAOAB, full-range forces (comparator)
    ns_day_b = ms_b = pairs_full = None
    prof_b = None
    if not a.no_baoab:
        split_b = S.water_split(r_s=5.0, r_c=a.rc, w=1.0, skin=a.baoab_skin, n_rings=a.rings)
        pb = params(False, a.graph_steps)
        bs = jumpmd.Sim(sysm, split_b, pb)
        dt_b = timed(bs, bstep(bs), a.steps, a.warmup)
        jumpmd.load().md_counters(bs._h, C.byref(pl), C.byref(pt))
        pairs_full = pl.value
        obs_b = bs.observables()
        bs.close()
        ms_b = 1e3 * dt_b / a.steps
        ns_day_b = n_sys * ns_per_day(step_ps, a.steps, dt_b)
        bp = jumpmd.Sim(sysm, split_b, params(False, 0))
        bstep(bp)(a.warmup)
        prof_b = kernel_profile(bp, bstep(bp), a.profile_steps)
        bp.close()
        print(f"[bench] {name_b} {ms_b:.4f} ms/step, {ns_day_b:.1f} ns/day, T = {obs_b['temperature']:.1f} K, "
              f"{pairs_full} pairs", flush=True)

    # dominant kernel of the JUMP step and its roofline
    dom = max(prof_j, key=lambda k: prof_j[k][0])
    tot_ms, launches = prof_j[dom]
    avg_s = tot_ms * 1e-3 / max(launches, 1)
    peak = PEAK_FP32_TFLOPS if prec else PEAK_FP64_TFLOPS
    if dom == 4:
        # one launch = one step's chains: proposals x algorithmic flops per proposal
        work = props_prof * FLOP_PER_PROPOSAL
        roof = {"bound": "alu", "achieved": work / avg_s / 1e12, "peak": peak, "unit": "TFLOP/s"}
    elif dom == 1:
        work = pairs_short * FLOP_PER_SHORT_PAIR
        roof = {"bound": "alu", "achieved": work / avg_s / 1e12, "peak": peak, "unit": "TFLOP/s"}
    else:
        work = n_atoms * BYTES_PER_ATOM_LOCAL
        roof = {"bound": "hbm", "achieved": work / avg_s / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = None
    if dom == 4 and (a.precision, a.n_mol, a.rings, a.skin, a.eps0, a.replicas, a.respa,
                     a.rc) == CHAIN_TRAFFIC["workload"]:
        import hashlib
        h = hashlib.sha256()
        for f in ("md_chain.hip", "md_device.h"):
            with open(os.path.join(ROOT, "paper_2412_15073_amd", "csrc", f), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest().startswith(CHAIN_TRAFFIC["sha256"]):
            roof["traffic"] = CHAIN_TRAFFIC["bytes"]
    roof["kernel"] = KERNELS[dom]
    roof["avg_launch_us"] = avg_s * 1e6
    roof["launches"] = launches

    def per_step(prof):
        return {KERNELS[k]: round(prof[k][0] / a.profile_steps, 5) for k in prof if prof[k][1]}

    # CPU baseline: the oracle, single thread, on a bounded sample of the same workload
    cpu = None
    if not a.no_cpu_baseline:
        from oracle.oracle import OracleSim
        po = params(True, 0)
        osys = sysm.systems[0] if a.replicas else sysm
        o = OracleSim(osys, split, po)
        ostep = o.step_jump_respa if a.respa else o.step_jump
        ostep(1)   # untimed: builds the oracle's rows
        # timed: whole steps until the budget is spent
        n_more, t = 0, time.perf_counter()
        while True:
            ostep(1)
            n_more += 1
            el = time.perf_counter() - t
            if el >= a.cpu_seconds:
                break
        cpu = {"value": ns_per_day(step_ps, n_more, el), "unit": "ns/day", "cores": 1, "kind": "oracle",
               "sample": f"{n_more} {name_j} steps of {'replica 0 of the ensemble, ' if a.replicas else 'the same '}"
                         f"{osys.n_atoms}-atom water system, after 1 untimed step (brute-force O(N^2) pair sums, "
                         f"single thread), {el:.1f} s"}
        print(f"[bench] oracle {el / n_more:.3f} s/step", flush=True)

    line = {
        "metric": "ns/day & pair-interactions/s, JUMP vs full-force BAOAB, 1 MI355X, matched T/RDF/D",
        "value": ns_day_j, "unit": "ns/day", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms_j, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == 0 else "f32+f64", "data": "synthetic (lattice water, BAOAB-equilibrated, seeded)",
        "config": {"workload": (f"water_{a.replicas}replicas_jump_{a.precision}" if a.replicas else
                                f"water_{a.n_mol}mol_jump{'_respa' if a.respa else ''}_{a.precision}"),
                   "n_atoms": n_atoms,
                   "box_A": None if a.replicas else round(float(sysm.box[0]), 3), "r_s": 5.0, "r_c": a.rc,
                   "switch": 1.0, "respa_inner": a.respa_inner if a.respa else None,
                   "skin": a.skin, "baoab_skin": a.baoab_skin, "rings": a.rings, "dt_fs": 1.0, "gamma_per_ps": 1.0, "T_K": 300,
                   "eps0_per_kcal_mol_A": a.eps0, "jumps": "LJ BPS + Coulomb adaptive MRZ",
                   "chain_lanes": a.chain_lanes, "graph_steps": a.graph_steps},
        "baoab_full_ns_per_day": ns_day_b, "baoab_full_ms_per_step": ms_b,
        "jump_speedup_vs_baoab": (ns_day_j / ns_day_b) if ns_day_b else None,
        "pair_interactions_per_s": {
            "work": (pairs_short + props) * a.steps / dt_j,
            "effective": (pairs_full * a.steps / dt_j) if pairs_full else None,
            "baoab_full": (pairs_full * 1e3 / ms_b) if pairs_full else None},
        "proposals_per_step": props, "short_pairs": pairs_short, "full_pairs": pairs_full,
        "kernel_ms_per_step": per_step(prof_j),
        "baoab_kernel_ms_per_step": per_step(prof_b) if prof_b else None,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
