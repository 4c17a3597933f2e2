#!/usr/bin/env python
"""Throughput of the JUMP hot path on one MI355X, with full-range BAOAB beside it.

Headline workload (default): the batched ensemble. 256 independent water
replicas whose sizes are drawn uniformly from 216-2048 molecules (seed 1;
box edges for 0.0334 molecules/A^3, 18.6-39.4 A), 869k atoms in all, in one
context: every kernel launch covers all replicas and the JUMP steps replay as
captured HIP graphs. JUMP (C' J' A O A J' C': short forces below r_s = 5 A with
a 1 A switch, the long part out to r_c = 10 A as jumps: LJ BPS, Coulomb
adaptive MRZ with eps0 = 0.1 (kcal/mol/A)^-1) runs FP32-mixed (pair forces
and jump rates in FP32, FP64 state and sums); the comparator is plain FP64
BAOAB with full-range forces (r < r_c). Replicas with an edge below
2 (r_c + skin) keep explicit periodic images in their rows. dt = 1 fs,
gamma = 1/ps, 300 K. `value` is the aggregate ns/day over all replicas.

Further workloads of the same line (key "workloads"), each with its own
comparator, kernel split and roofline:
  water4096        4096 waters (12288 atoms, 49.7 A), FP64 JUMP vs FP64 BAOAB;
  water4096_fp32   the same system, FP32-mixed JUMP vs the FP64 BAOAB above;
  water32000_respa 32000 waters (96000 atoms, 98.6 A), r_c = 12 A, JUMP-RESPA
                   (bonded forces every 1 fs, short forces and jumps every
                   3 fs) FP32-mixed vs FP64 BAOAB-RESPA with full forces;
  water4096_pme_respa1  the 4096-water box with the paper's Ewald settings
                   for its 12 000-atom water (damped real part to 7 A with
                   alpha 0.554 A^-1, jumps between r_s = 5 A (switch 0.5 A) and
                   7 A, the reciprocal sum by particle-mesh Ewald on a 64^3
                   mesh, order 6): JUMP-RESPA1 at 1:2:6 fs (bonded 1 fs, short
                   forces and jumps 2 fs, reciprocal forces 6 fs) FP32-mixed vs
                   FP64 BAOAB-RESPA1 at the same steps;
  water4096_pme_matched  the 4096-water box at the same Ewald settings, plain
                   JUMP (reciprocal forces every step in the C' acceleration)
                   at the cheapest point of the accuracy frontier that keeps
                   T within 1 %, the O-O RDF within 1e-2 and D within 5 % of
                   FP64 BAOAB: r_s = 6 A, eps0 = 0.1, the LJ long part jumping
                   in the C step with the Coulomb part; FP32-mixed JUMP vs
                   FP64 BAOAB (full forces to 7 A + PME every step);
  lj864            864 LJ atoms (fcc, rho 0.8442, kT 0.722), B J A O A J B with
                   BPS jumps between r_s = 3 and r_c = 5 sigma, vs BAOAB, FP64
                   (reduced units: tau/day).

Inputs are synthetic (lattice start, then an untimed BAOAB equilibration);
everything timed is resident in HBM. Timed region: K steps (HIP graphs of
--graph-steps steps where the scheme allows), bracketed by synchronisations.
Per-kernel durations for the roofline come from a second, profiled run of
plain launches in the same process (HIP events on the library's stream).

CPU baseline: the oracle (plain FP64 C, single-threaded per process) on a
stratified sample of the ensemble's replicas, one replica per host core in
parallel processes; the whole-ensemble rate is estimated from the mean
per-step time of the sample.

Prints ONE JSON line. --gpus N > 1 exits: the benchmark runs on one GPU.
"""
import argparse
import json
import os
import subprocess
import sys
import tempfile
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
#  particle-mesh Ewald, per evaluation: spreading (a product of three
#  weights per grid point, 3 flops) and gathering (three products and three
#  fmas per grid point, 9 flops) over p^3 points per atom, plus two complex
#  three-dimensional transforms of 5 N log2 N flops each and the influence
#  function (6 flops per grid point).
FLOP_PME_SPREAD_GATHER = 12
FLOP_PME_POINT = 6
BYTES_PER_ATOM_LOCAL = 7 * 32   # x (read+write), v (read+write), f_nb, f_b, x_ref reads
# one row build: per atom, binning (x read, reference copy written, cell index
# and slot), scatter (cell-ordered FP64 and FP32 position copies) and the
# builder's own reads, about 200 B; plus 4 B per row entry and per segment start written
BYTES_PER_ATOM_BUILD = 200
BYTES_PER_ROW_ENTRY = 4
# HBM bytes of the chain kernel per proposal, from FETCH_SIZE / WRITE_SIZE
# counters per launch (each scaled by the same counter on a plain 256 MiB
# copy: fetch x 1.9998, write x 1.0) divided by that launch's proposals
# (summaries under profiles/), per workload, valid while the sha256 of the
# chain kernel's sources (md_chain.hip, then md_device.h) starts with the
# given prefix. The line reports it times the proposals of its own launches.
CHAIN_TRAFFIC = {
    "ensemble": {"sha256": "284d8ca1b862a64f", "bytes_per_proposal": 241.9},
    "water4096": {"sha256": "284d8ca1b862a64f", "bytes_per_proposal": 46.9},
}
KERNELS = {0: "k_local (B/A/O updates)", 1: "k_force (pairs, with bonded when fused)", 2: "k_bonded (separate)",
           3: "row rebuild", 4: "k_chain (J/C jump chains)", 5: "reciprocal space (particle-mesh Ewald)"}
METRIC = "ns/day & pair-interactions/s, JUMP vs full-force BAOAB, 1 MI355X, matched T/RDF/D"
ALL_WORKLOADS = ("ensemble", "water4096", "water4096_fp32", "water32000_respa", "water4096_pme_respa1",
                 "water4096_pme_matched", "lj864")
PME = {"alpha": 0.554, "r_s": 5.0, "r_c": 7.0, "switch": 0.5, "grid": 64, "order": 6}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--equil", type=int, default=4000, help="untimed BAOAB steps at 0.5 fs, gamma 10/ps (water)")
    ap.add_argument("--workloads", default=",".join(ALL_WORKLOADS),
                    help="comma list; the first is the headline (value, roofline, cpu_baseline)")
    ap.add_argument("--replicas", type=int, default=256, help="replicas of the ensemble")
    ap.add_argument("--eps0", type=float, default=0.1, help="adaptive eps0 in (kcal/mol/A)^-1")
    ap.add_argument("--rings", type=int, default=12)
    ap.add_argument("--skin", type=float, default=0.5)
    ap.add_argument("--baoab-skin", type=float, default=1.0,
                    help="list skin of the BAOAB comparator (its fastest; JUMP's fastest is 0.5)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget per process of the oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--chain-lanes", type=int, default=0, help="lanes per atom in the jump chains (0 = auto)")
    ap.add_argument("--chain-order", type=int, default=0, help="wave order of the chains (0 auto, 1 type, 2 replica)")
    ap.add_argument("--graph-steps", type=int, default=20, help="steps per replayed HIP graph (0 = plain launches)")
    ap.add_argument("--profile-steps", type=int, default=200, help="plain-launch steps timed per kernel")
    ap.add_argument("--no-baoab", action="store_true", help="skip the comparators (profiling runs)")
    ap.add_argument("--no-tune", action="store_true", help="ensemble: default settings instead of md_tune's")
    ap.add_argument("--tune-steps", type=int, default=40, help="timed steps per autotuner trial")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (HBM counter calibration) and exit")
    ap.add_argument("--cpu-worker", default="", help=argparse.SUPPRESS)
    return ap.parse_args()


# ------------------------------------------------------------------ CPU side
def cpu_worker(spec):
    """One process of the CPU baseline (never touches the GPU): the oracle on
    one replica of the ensemble from the equilibrated state in `spec`
    (npz path:replica index), whole JUMP steps until the budget is spent."""
    import numpy as np
    from oracle.oracle import OracleSim
    from paper_2412_15073_amd import systems as S
    path, r, seconds, eps0, rings, skin = spec.split(":")
    d = np.load(path)
    r = int(r)
    sy = S.water_box(int(d[f"nmol_{r}"]), seed=int(d[f"seed_{r}"]))
    sy.pos, sy.vel = d[f"x_{r}"], d[f"v_{r}"]
    split = S.water_split(r_s=5.0, r_c=10.0, w=1.0, skin=float(skin), n_rings=int(rings))
    pa = S.water_params(eps0_per_kcal=float(eps0))
    o = OracleSim(sy, split, pa, replica=r)
    o.step_jump(1)   # untimed: builds the oracle's rows
    n, t = 0, time.perf_counter()
    while True:
        o.step_jump(1)
        n += 1
        el = time.perf_counter() - t
        if el >= float(seconds):
            break
    print(json.dumps({"replica": r, "n_atoms": sy.n_atoms, "steps": n, "seconds": el}), flush=True)


def host_cores():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline_ensemble(a, batch, x, v, n_rep):
    """Oracle on a stratified sample of replicas (every n_rep/C-th by index),
    C processes in parallel, one per host core."""
    import numpy as np
    cores = host_cores()
    from paper_2412_15073_amd import systems as S
    recipe = S.water_replica_recipe(n_rep, n_min=216, seed=1)
    picks = sorted(set(int(round(k * n_rep / cores)) % n_rep for k in range(cores)))
    data = {}
    for r in picks:
        lo, hi = batch.offsets[r], batch.offsets[r + 1]
        data[f"x_{r}"], data[f"v_{r}"] = x[lo:hi], v[lo:hi]
        data[f"nmol_{r}"] = np.array(recipe[r][0])
        data[f"seed_{r}"] = np.array(recipe[r][1])
    fd, path = tempfile.mkstemp(suffix=".npz")
    os.close(fd)
    np.savez(path, **data)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    t0 = time.perf_counter()
    procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker",
                               f"{path}:{r}:{a.cpu_seconds}:{a.eps0}:{a.rings}:{a.skin}"],
                              stdout=subprocess.PIPE, stderr=subprocess.PIPE, env=env, cwd=ROOT) for r in picks]
    res = []
    for p in procs:
        out, err = p.communicate()
        if p.returncode != 0:
            raise RuntimeError(f"cpu worker failed: {err.decode()[-2000:]}")
        res.append(json.loads(out.decode().strip().splitlines()[-1]))
    wall = time.perf_counter() - t0
    os.remove(path)
    per_step = [q["seconds"] / q["steps"] for q in res]
    mean_t = sum(per_step) / len(per_step)
    # a whole-ensemble step on C cores takes sum_r t_r / C = n_rep * mean_t / C;
    # every replica advances 1 fs = 1e-6 ns per step
    value = 1e-6 * 86400.0 * len(res) / mean_t
    return {"value": value, "unit": "ns/day", "cores": len(res), "kind": "oracle",
            "single_core_value": 1e-6 * 86400.0 / mean_t,
            "sample": (f"oracle (FP64 C, one thread per process) on {len(res)} of the {n_rep} replicas "
                       f"(every {n_rep / len(res):.0f}th by index, {min(q['n_atoms'] for q in res)}-"
                       f"{max(q['n_atoms'] for q in res)} atoms) in {len(res)} parallel processes, "
                       f"{sum(q['steps'] for q in res)} JUMP steps in {wall:.1f} s wall after 1 untimed step "
                       f"each; whole-ensemble rate = cores x 1 fs / mean per-step time "
                       f"({1e3 * mean_t:.1f} ms)")}


# ------------------------------------------------------------------ GPU side
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


def chain_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("md_chain.hip", "md_device.h"):
        with open(os.path.join(ROOT, "paper_2412_15073_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


class Workload:
    """One benchmark workload: system, split, schemes, precision, units."""

    def __init__(self, name, a, S):
        self.name = name
        self.respa = name == "water32000_respa"
        self.respa1 = name == "water4096_pme_respa1"
        self.matched = name == "water4096_pme_matched"
        self.pme = self.respa1 or self.matched
        self.lj = name == "lj864"
        self.ensemble = name == "ensemble"
        self.jump_prec = {"ensemble": 1, "water4096": 0, "water4096_fp32": 1, "water32000_respa": 1,
                          "water4096_pme_respa1": 1, "water4096_pme_matched": 1, "lj864": 0}[name]
        self.rc = 12.0 if self.respa else (PME["r_c"] if self.pme else 10.0)
        self.rs = 6.0 if self.matched else (3.0 if self.lj else 5.0)
        self.inner = 3 if self.respa else (2 if self.respa1 else 1)
        self.outer = 3 if self.respa1 else 1
        self.graph = 0 if (self.respa or self.respa1) else a.graph_steps
        self.S = S
        self.a = a
        if self.ensemble:
            self.system = lambda: S.water_replicas(a.replicas, n_min=216, seed=1)
            self.n_sys = a.replicas
        elif self.lj:
            self.system = lambda: S.lj_fcc(6, seed=1)
            self.n_sys = 1
        else:
            n_mol = 32000 if self.respa else 4096
            self.system = lambda: S.water_box(n_mol, seed=1)
            self.n_sys = 1
        self.step_unit = 0.005 if self.lj else 1e-6 * self.inner * self.outer   # simulated tau, or ns, per call step

    def split(self, skin):
        if self.lj:
            return self.S.lj_split(skin=0.3)
        if self.pme:
            sp = self.S.water_split(r_s=self.rs, r_c=self.rc, w=PME["switch"], skin=skin, alpha=PME["alpha"],
                                    n_rings=6)
            sp.coulomb_kind, sp.pme_grid, sp.pme_order = self.S.COUL_SPME, (PME["grid"],) * 3, PME["order"]
            return sp
        return self.S.water_split(r_s=5.0, r_c=self.rc, w=1.0, skin=skin, n_rings=self.a.rings)

    def params(self, jumps, prec, graph):
        S = self.S
        if self.lj:
            p = S.lj_params(seed=2, jumps=jumps)
        else:
            p = S.water_params(eps0_per_kcal=self.a.eps0, jumps=jumps)
            if self.respa or self.respa1:
                p.respa_inner = self.inner
                p.respa_outer = self.outer
            if self.matched and jumps:
                p.jump_lj = S.JUMP_IN_C
        p.chain_lanes = self.a.chain_lanes
        p.chain_order = self.a.chain_order
        p.graph_steps = graph
        p.precision = prec
        return p

    def equilibrate(self, jumpmd, sysm):
        S, a = self.S, self.a
        if self.lj:
            eq = jumpmd.Sim(sysm, self.split(0.3), S.lj_params(jumps=False))
            eq.step_baoab(10000)
        else:
            eq = jumpmd.Sim(sysm, self.split(1.0), S.water_params(dt=0.0005, gamma=10.0, jumps=False))
            eq.step_baoab(a.equil)
        T = eq.observables()["temperature"]
        x, v = eq.state()
        eq.close()
        return x, v, T


def set_state(sy, x, v):
    if hasattr(sy, "systems"):
        for r, s_r in enumerate(sy.systems):
            lo, hi = sy.offsets[r], sy.offsets[r + 1]
            s_r.pos, s_r.vel = x[lo:hi], v[lo:hi]
    else:
        sy.pos, sy.vel = x, v


def pme_flops(n_atoms, grid, order):
    """Algorithmic flops of one particle-mesh Ewald evaluation."""
    import math
    ng = grid ** 3
    return (n_atoms * order ** 3 * FLOP_PME_SPREAD_GATHER + 2 * 5 * ng * math.log2(ng) + FLOP_PME_POINT * ng)


def roofline(prof, steps_prof, props_prof, pairs_short, n_atoms, prec, build_bytes_prof=0.0, pme_work=0.0):
    dom = max(prof, key=lambda k: prof[k][0])
    tot_ms, launches = prof[dom]
    avg_s = tot_ms * 1e-3 / max(launches, 1)
    peak = PEAK_FP32_TFLOPS if prec else PEAK_FP64_TFLOPS
    if dom == 4:
        # one launch = one (outer) step's chains: proposals x algorithmic flops per proposal
        work = props_prof * FLOP_PER_PROPOSAL * steps_prof / max(launches, 1)
        roof = {"bound": "alu", "achieved": work / avg_s / 1e12, "peak": peak, "unit": "TFLOP/s",
                "algorithmic": f"{FLOP_PER_PROPOSAL} flop/proposal x {work / FLOP_PER_PROPOSAL:.0f} proposals/launch"}
    elif dom == 1:
        work = pairs_short * FLOP_PER_SHORT_PAIR
        roof = {"bound": "alu", "achieved": work / avg_s / 1e12, "peak": peak, "unit": "TFLOP/s",
                "algorithmic": f"{FLOP_PER_SHORT_PAIR} flop/pair x {pairs_short} pairs/launch"}
    elif dom == 5:
        # one evaluation: spreading, two transforms, influence function, gathering, FP64
        work = pme_work
        roof = {"bound": "alu", "achieved": work / avg_s / 1e12, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "algorithmic": f"{work:.3g} flop per evaluation (spread/gather {FLOP_PME_SPREAD_GATHER} flop x "
                               f"order^3 per atom, 2 transforms x 5 N log2 N, {FLOP_PME_POINT} flop per mesh point)"}
    elif dom == 3:
        # every step launches the displacement check; builds happen on some steps
        work = build_bytes_prof / max(launches, 1)
        roof = {"bound": "hbm", "achieved": work / avg_s / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "algorithmic": f"{BYTES_PER_ATOM_BUILD} B/atom + {BYTES_PER_ROW_ENTRY} B/row entry per build, "
                               f"{work:.0f} B/launch averaged over {launches} launches"}
    else:
        work = n_atoms * BYTES_PER_ATOM_LOCAL
        roof = {"bound": "hbm", "achieved": work / avg_s / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "algorithmic": f"{BYTES_PER_ATOM_LOCAL} B/atom x {n_atoms} atoms"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = None
    roof["kernel"] = KERNELS[dom]
    roof["avg_launch_us"] = avg_s * 1e6
    roof["launches"] = launches
    return dom, roof


def run_workload(w, jumpmd, C, cache):
    """Times JUMP and its comparator on one workload; returns (result, state)."""
    a = w.a
    sysm = w.system()
    n_atoms = int(sysm.offsets[-1]) if w.ensemble else sysm.n_atoms
    t = time.perf_counter()
    key = "water4096" if w.name.startswith("water4096") else w.name
    if key in cache:
        x, v, T_eq = cache[key]["state"]
    else:
        x, v, T_eq = w.equilibrate(jumpmd, sysm)
    print(f"[bench] {w.name}: {n_atoms} atoms, equilibrated in {time.perf_counter() - t:.1f} s, T = {T_eq:.1f}",
          flush=True)
    set_state(sysm, x, v)
    jstep = (lambda s: s.step_jump_respa) if w.respa else (
        (lambda s: s.step_jump_respa1) if w.respa1 else (lambda s: s.step_jump))
    bstep = (lambda s: s.step_baoab_respa) if w.respa else (
        (lambda s: s.step_baoab_respa1) if w.respa1 else (lambda s: s.step_baoab))
    split_j = w.split(a.skin)
    pj = w.params(True, w.jump_prec, w.graph)
    tuned = None
    if w.ensemble and not a.no_tune:
        # autotuned lanes, skin, rings and graph replay (md_tune), outside the timed region
        t = time.perf_counter()
        split_j, pj, ms_t, trials = jumpmd.tune(sysm, split_j, pj, scheme="jump_respa" if w.respa else "jump",
                                                steps=a.tune_steps)
        tuned = {"jump": {"chain_lanes": pj.chain_lanes, "chain_order": pj.chain_order, "skin": split_j.skin,
                          "rings": split_j.n_rings,
                          "graph_steps": pj.graph_steps, "trials": len(trials), "ms_per_step": ms_t}}
        print(f"[bench] {w.name} JUMP tuned in {time.perf_counter() - t:.1f} s: {tuned['jump']}", flush=True)
    pl, pt = C.c_int64(0), C.c_int64(0)

    js = jumpmd.Sim(sysm, split_j, pj)
    p0 = js.proposals_total()
    dt_j = timed(js, jstep(js), a.steps, a.warmup)
    props = (js.proposals_total() - p0) / (a.steps + a.warmup)
    obs_j = js.observables()
    jumpmd.load().md_counters(js._h, C.byref(pl), C.byref(pt))
    pairs_short = pl.value
    xj, vj = js.state()
    js.close()
    ms_j = 1e3 * dt_j / a.steps
    rate_j = w.n_sys * w.step_unit * a.steps / dt_j * 86400.0

    s2 = w.system()
    set_state(s2, xj, vj)
    pj0 = w.params(True, w.jump_prec, 0)
    pj0.chain_lanes, pj0.chain_order = pj.chain_lanes, pj.chain_order
    jp = jumpmd.Sim(s2, split_j, pj0)
    jstep(jp)(min(a.warmup, 20))
    q0 = jp.proposals_total()
    nb0 = jp.observables()["n_rebuilds"]
    prof_j = kernel_profile(jp, jstep(jp), a.profile_steps)
    props_prof = (jp.proposals_total() - q0) / a.profile_steps
    # algorithmic bytes of the row builds in the profiled window: replica builds
    # times the bytes of an average replica's build (short + candidate rows)
    builds = jp.observables()["n_rebuilds"] - nb0
    entries = int(jp.row_counts(0).sum()) + int(jp.row_counts(2).sum())
    n_seg = (1 if w.lj else split_j.n_rings) * (1 if w.lj else 2)
    build_bytes = builds / w.n_sys * (BYTES_PER_ATOM_BUILD * n_atoms + BYTES_PER_ROW_ENTRY * (entries + n_atoms * (n_seg + 1)))
    jp.close()
    unit = "tau/day" if w.lj else "ns/day"
    print(f"[bench] {w.name} JUMP {ms_j:.4f} ms/step, {rate_j:.1f} {unit}, T = {obs_j['temperature']:.1f}, "
          f"{props:.0f} proposals/step", flush=True)

    # comparator: FP64 BAOAB (or BAOAB-RESPA) with full-range forces
    base = None
    if not a.no_baoab:
        if w.name == "water4096_fp32" and cache.get("baoab:water4096"):
            base = cache["baoab:water4096"]
        else:
            split_b = w.split(0.3 if w.lj else a.baoab_skin)
            pb = w.params(False, 0, w.graph)
            if w.ensemble and not a.no_tune:
                t = time.perf_counter()
                split_b, pb, ms_t, trials = jumpmd.tune(sysm, split_b, pb,
                                                        scheme="baoab_respa" if w.respa else "baoab",
                                                        steps=a.tune_steps)
                tuned["baoab"] = {"skin": split_b.skin, "graph_steps": pb.graph_steps, "trials": len(trials),
                                  "ms_per_step": ms_t}
                print(f"[bench] {w.name} BAOAB tuned in {time.perf_counter() - t:.1f} s: {tuned['baoab']}",
                      flush=True)
            bs = jumpmd.Sim(sysm, split_b, pb)
            dt_b = timed(bs, bstep(bs), a.steps, a.warmup)
            jumpmd.load().md_counters(bs._h, C.byref(pl), C.byref(pt))
            pairs_full = pl.value
            obs_b = bs.observables()
            bs.close()
            bp = jumpmd.Sim(sysm, split_b, w.params(False, 0, 0))
            bstep(bp)(min(a.warmup, 20))
            prof_b = kernel_profile(bp, bstep(bp), a.profile_steps)
            bp.close()
            ms_b = 1e3 * dt_b / a.steps
            base = {"ms_per_step": ms_b, "rate": w.n_sys * w.step_unit * a.steps / dt_b * 86400.0,
                    "skin": split_b.skin,
                    "full_pairs": pairs_full, "T": obs_b["temperature"],
                    "kernel_ms_per_step": {KERNELS[k]: round(prof_b[k][0] / a.profile_steps, 5)
                                           for k in prof_b if prof_b[k][1]}}
            print(f"[bench] {w.name} BAOAB FP64 {ms_b:.4f} ms/step, {base['rate']:.1f} {unit}, "
                  f"T = {obs_b['temperature']:.1f}, {pairs_full} pairs", flush=True)

    pme_work = pme_flops(n_atoms, PME["grid"], PME["order"]) if w.pme else 0.0
    dom, roof = roofline(prof_j, a.profile_steps, props_prof, pairs_short, n_atoms, w.jump_prec, build_bytes, pme_work)
    tr = CHAIN_TRAFFIC.get(w.name)
    if dom == 4 and tr and chain_source_hash().startswith(tr["sha256"]):
        roof["traffic"] = tr["bytes_per_proposal"] * props_prof * a.profile_steps / max(roof["launches"], 1)
    steps_per_day = a.steps / dt_j * 86400.0
    res = {
        "workload": w.name, "n_atoms": n_atoms, "replicas": w.n_sys,
        "jump_precision": "fp32-mixed" if w.jump_prec else "fp64", "comparator_precision": "fp64",
        "ms_per_step": ms_j, unit.replace("/", "_per_"): rate_j, "T_K_or_kT": obs_j["temperature"],
        "baoab_ms_per_step": base["ms_per_step"] if base else None,
        "baoab_" + unit.replace("/", "_per_"): base["rate"] if base else None,
        "jump_speedup_vs_baoab": (rate_j / base["rate"]) if base else None,
        "proposals_per_step": props, "short_pairs": pairs_short,
        "full_pairs": base["full_pairs"] if base else None,
        "pair_interactions_per_s": {
            "work": (pairs_short + props) * steps_per_day / 86400.0,
            "effective": (base["full_pairs"] * steps_per_day / 86400.0) if base else None,
            "baoab_full": (base["full_pairs"] * 1e3 / base["ms_per_step"]) if base else None},
        "kernel_ms_per_step": {KERNELS[k]: round(prof_j[k][0] / a.profile_steps, 5) for k in prof_j if prof_j[k][1]},
        "baoab_kernel_ms_per_step": base["kernel_ms_per_step"] if base else None,
        "roofline": roof,
        "config": {"r_s": w.rs, "r_c": 5.0 if w.lj else w.rc,
                   "switch": 0.5 if (w.lj or w.pme) else 1.0,
                   "skin": 0.3 if w.lj else split_j.skin, "baoab_skin": base["skin"] if base else None,
                   "rings": 1 if w.lj else split_j.n_rings, "chain_lanes": pj.chain_lanes, "autotuned": tuned,
                   "respa_inner": w.inner if (w.respa or w.respa1) else None,
                   "respa_outer": w.outer if w.respa1 else None,
                   "electrostatics": (f"particle-mesh Ewald (alpha {PME['alpha']}, {PME['grid']}^3 mesh, order "
                                      f"{PME['order']})" if w.pme else (None if w.lj else "DSF (alpha 0.2)")),
                   "dt": "0.005 tau" if w.lj else "1 fs", "graph_steps": pj.graph_steps,
                   "eps0_per_kcal_mol_A": None if w.lj else a.eps0,
                   "jumps": "LJ BPS" if w.lj else ("LJ and Coulomb long parts, adaptive MRZ in the C step" if w.matched
                                                   else "LJ BPS + Coulomb adaptive MRZ")},
    }
    cache[key] = {"state": (x, v, T_eq)}
    cache["baoab:" + w.name] = base
    return res, (sysm, x, v)


def main():
    a = parse()
    if a.cpu_worker:
        cpu_worker(a.cpu_worker)
        return
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

    names = [n for n in a.workloads.split(",") if n]
    for n in names:
        if n not in ALL_WORKLOADS:
            raise SystemExit(f"unknown workload {n}; choose from {ALL_WORKLOADS}")
    cache, results, head_state = {}, {}, None
    for n in names:
        w = Workload(n, a, S)
        results[n], st = run_workload(w, jumpmd, C, cache)
        if n == names[0]:
            head_state = (w, st)
    head = results[names[0]]
    w0, (sys0, x0, v0) = head_state

    cpu = None
    if not a.no_cpu_baseline and w0.ensemble:
        cpu = cpu_baseline_ensemble(a, sys0, x0, v0, w0.n_sys)
        print(f"[bench] oracle: {cpu['value']:.4f} ns/day on {cpu['cores']} cores", flush=True)

    unit = "tau/day" if w0.lj else "ns/day"
    ukey = unit.replace("/", "_per_")
    line = {
        "metric": METRIC,
        "value": head[ukey], "unit": unit, "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if w0.jump_prec else "f64",
        "data": "synthetic (lattice water, BAOAB-equilibrated, seeded)",
        "config": {"workload": {"ensemble": f"water_ensemble_{w0.n_sys}replicas_216-2048mol_jump_fp32mixed"}.get(
                       names[0], names[0]), "n_atoms": head["n_atoms"], "replicas": head["replicas"],
                   "comparator": "FP64 BAOAB, full-range forces", **head["config"]},
        "baoab_full_ns_per_day": head.get("baoab_" + ukey), "baoab_full_ms_per_step": head["baoab_ms_per_step"],
        "jump_speedup_vs_baoab": head["jump_speedup_vs_baoab"],
        "pair_interactions_per_s": head["pair_interactions_per_s"],
        "proposals_per_step": head["proposals_per_step"], "short_pairs": head["short_pairs"],
        "full_pairs": head["full_pairs"],
        "kernel_ms_per_step": head["kernel_ms_per_step"],
        "baoab_kernel_ms_per_step": head["baoab_kernel_ms_per_step"],
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
        "workloads": {n: results[n] for n in names[1:]},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
