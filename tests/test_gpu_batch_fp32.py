"""Batched replicas and the FP32-mixed path on the GPU.

Batched: each replica of a batch, advanced in the same launches, must give
exactly the oracle run of that replica alone (its random streams are keyed
by the replica index). FP32-mixed: pair forces and jump rates in FP32 with
FP64 accumulation; forces must match the FP64 oracle to FP32 accuracy and
the jump steps must still reproduce the long-range force on average.
"""
import numpy as np
import pytest
import scipy.stats as st

from paper_2412_15073_amd import systems as S
from tests.helpers import water_small, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def jm():
    from paper_2412_15073_amd import jumpmd
    jumpmd.load()
    return jumpmd


def _batch():
    sizes = [96, 125, 150]
    systems = [S.water_box(m, seed=20 + r, jitter=0.05) for r, m in enumerate(sizes)]
    sp = S.water_split(r_s=5.0, r_c=7.0, w=1.0, skin=0.5, n_rings=3)
    return S.Batch(systems), sp


@pytest.mark.parametrize("scheme", ["jump", "baoab", "jump_respa", "jump_bps"])
def test_batched_replicas_match_single_replica_oracle(jm, scheme):
    from oracle.oracle import OracleSim
    batch, sp = _batch()
    pa = S.water_params(jumps=(scheme != "baoab"))
    if scheme == "jump_bps":
        pa.jump_coul = S.JUMP_BPS
    pa.log_events = 1
    pa.respa_inner = 3
    g = jm.Sim(batch, sp, pa)
    run = {"jump": "step_jump", "baoab": "step_baoab", "jump_respa": "step_jump_respa",
           "jump_bps": "step_jump"}[scheme]
    getattr(g, run)(6)
    xg, vg = g.state()
    sg = g.atom_stats()
    evg = g.events()
    off = batch.offsets
    for r, sysr in enumerate(batch.systems):
        o = OracleSim(sysr, sp, pa, replica=r)
        getattr(o, run)(6)
        xo, vo = o.state()
        a, b = off[r], off[r + 1]
        assert rel_err(xg[a:b], xo) < 1e-9 and rel_err(vg[a:b], vo) < 1e-9, r
        so = o.atom_stats()
        for k in ("n_prop", "n_acc", "hash"):
            np.testing.assert_array_equal(sg[k][a:b], so[k], err_msg=f"replica {r} {k}")
        if scheme != "baoab":
            mine = evg[(evg[:, 2] >= a) & (evg[:, 2] < b)].copy()
            mine[:, 2] -= a
            mine[:, 3] -= a
            np.testing.assert_array_equal(mine, o.events())


def test_batched_replica_rows_match(jm):
    from oracle.oracle import OracleSim
    batch, sp = _batch()
    g = jm.Sim(batch, sp, S.water_params())
    off = batch.offsets
    for r, sysr in enumerate(batch.systems):
        o = OracleSim(sysr, sp, S.water_params(), replica=r)
        o.build_lists()
        for i in range(0, sysr.n_atoms, 5):
            jg, sg = g.cand_row(off[r] + i, o.n_segments)
            np.testing.assert_array_equal(jg - off[r], o.cand_row(i))
            np.testing.assert_array_equal(sg, o.seg_start(i))


def test_fp32_forces_match_fp64_oracle(jm):
    from oracle.oracle import OracleSim, F_SHORT, F_FULL
    sy, sp = water_small()
    pa = S.water_params()
    pa.precision = S.FP32_MIXED
    g = jm.Sim(sy, sp, pa)
    o = OracleSim(sy, sp, S.water_params())
    # FP32 pair terms: a few ulp of float per pair, summed over ~100 pairs
    assert rel_err(g.accel(0), o.accel(F_SHORT)) < 2e-5
    assert rel_err(g.accel(1), o.accel(F_FULL)) < 2e-5


@pytest.mark.parametrize("kind", [S.JUMP_MRZ_ADAPTIVE, S.JUMP_BPS])
@pytest.mark.parametrize("precision", [S.FP64, S.FP32_MIXED])
def test_gpu_c_step_mean_kick_equals_long_force(jm, precision, kind):
    """Generator-moment identity run on the GPU path: from Maxwell-Boltzmann
    velocities the C step changes v by -h grad U_long / m on average (ion
    lattice, short force exactly zero), in FP64 and with FP32 rates, for the
    adaptive MRZ jumps and for the BPS bounces."""
    from oracle.oracle import OracleSim, F_FULL
    sy = S.ion_lattice(4, 3.3, jitter=0.1, neutral_every=5)
    sp = S.Split(r_s=3.0, r_c=5.0, switch_width=1.0, skin=0.3, coulomb_alpha=0.2, n_rings=3,
                 ring_width=(5.3 - 1.7) / 3)
    pa = S.Params(dt=0.01, gamma=0.0, kT=1.0, jump_coul=kind, eps=0.3, precision=precision)
    g = jm.Sim(sy, sp, pa)
    h, K = 0.05, 6000
    expected = h * OracleSim(sy, sp, S.Params(dt=0.01, gamma=0.0, kT=1.0, jump_coul=S.JUMP_MRZ_ADAPTIVE,
                                               eps=0.3)).accel(F_FULL)
    x0, v0 = g.state()
    rng = np.random.default_rng(3)
    dv = []
    for k in range(K):
        v = rng.standard_normal(v0.shape)
        g.set_state(vel=v, step=k)
        g.run_phase("C", "C1", h)
        dv.append(g.state()[1] - v)
    dv = np.array(dv)
    m, se = dv.mean(0), dv.std(0, ddof=1) / np.sqrt(K)
    live = se > 0
    z = (m - expected)[live] / se[live]
    z0 = m[live] / se[live]
    assert (z0 * z0).sum() > 10 * z.size
    assert st.chi2.sf((z * z).sum(), z.size) > 1e-3


@pytest.mark.parametrize("lanes", [0, 2])
def test_fp32_jump_run_is_stable_and_close(jm, lanes):
    """100 FP32-mixed JUMP steps: finite, same temperature and proposal rate
    as the FP64 path within statistical noise; automatic lanes, and 2 lanes
    per atom (the layout of large ensembles)."""
    sy, sp = water_small()
    out = {}
    for prec in (S.FP64, S.FP32_MIXED):
        pa = S.water_params()
        pa.precision = prec
        pa.chain_lanes = lanes
        g = jm.Sim(sy, sp, pa)
        g.step_jump(100)
        obs = g.observables(pe=True)
        out[prec] = obs
        assert np.isfinite(obs["ke"]) and obs["n_bound_viol"] <= obs["n_prop"] * 1e-6
    a, b = out[S.FP64], out[S.FP32_MIXED]
    assert abs(a["n_prop"] - b["n_prop"]) < 0.03 * a["n_prop"]
    assert abs(a["temperature"] - b["temperature"]) < 0.1 * a["temperature"]
