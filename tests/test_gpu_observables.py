"""GPU observables, the Z-sampler regimes and a 100-step water run against
the oracle (exact integers, FP64 values within 1e-9 relative)."""
import numpy as np
import pytest

from paper_2412_15073_amd import systems as S
from tests.helpers import water_small, rel_err

pytestmark = pytest.mark.gpu

TOL = 1e-9


@pytest.fixture(scope="module")
def jm():
    from paper_2412_15073_amd import jumpmd
    jumpmd.load()
    return jumpmd


def _pair(jm, system, split, params):
    from oracle.oracle import OracleSim
    return jm.Sim(system, split, params), OracleSim(system, split, params)


def _close(a, b, tol=TOL):
    return abs(a - b) <= tol * max(abs(b), 1e-300)


@pytest.mark.parametrize("scheme", ["jump", "baoab"])
def test_energies_and_temperature(jm, scheme):
    """Kinetic energy, temperature 2KE/(3N kB), and the potential energies of
    the split (short chi U, long (1 - chi) U, bonded) after 10 steps, from
    the rows the scheme keeps (short + candidate rows for JUMP, full rows for
    BAOAB), against the oracle's all-pairs sums."""
    sy, sp = water_small()
    pa = S.water_params(jumps=(scheme == "jump"))
    g, o = _pair(jm, sy, sp, pa)
    (g.step_jump if scheme == "jump" else g.step_baoab)(10)
    (o.step_jump if scheme == "jump" else o.step_baoab)(10)
    og, oo = g.observables(pe=True), o.energies()
    for kg, ko in (("ke", "ke"), ("temperature", "T"), ("pe_short", "pe_short"), ("pe_long", "pe_long"),
                   ("pe_bonded", "pe_bonded")):
        assert _close(og[kg], oo[ko]), (kg, og[kg], oo[ko])


def test_energies_of_every_replica(jm):
    """The same per replica of a batch of three uneven boxes: the batch's
    energies are the sums of the per-replica oracle values."""
    from oracle.oracle import OracleSim
    reps = [S.water_box(m, seed=10 + m, jitter=0.05) for m in (125, 180, 216)]
    sp = S.water_split(r_s=5.0, r_c=7.0, w=1.0, skin=0.5, n_rings=3)
    pa = S.water_params()
    g = jm.Sim(S.Batch(reps), sp, pa)
    g.step_jump(5)
    tot = {k: 0.0 for k in ("ke", "pe_short", "pe_long", "pe_bonded")}
    for r, sy in enumerate(reps):
        o = OracleSim(sy, sp, pa, replica=r)
        o.step_jump(5)
        e = o.energies()
        for k in tot:
            tot[k] += e[k]
    og = g.observables(pe=True)
    for k in tot:
        assert _close(og[k], tot[k]), (k, og[k], tot[k])


def test_rdf_counts(jm):
    """O-O, O-H and H-H pair-count histograms (r < 7.5 A, 0.05 A bins)
    identical to the oracle's after a few steps."""
    sy, sp = water_small()
    pa = S.water_params()
    g, o = _pair(jm, sy, sp, pa)
    g.step_jump(5)
    o.step_jump(5)
    for ta, tb in ((0, 0), (0, 1), (1, 1)):
        hg, ho = g.rdf_counts(ta, tb, 7.5, 150), o.rdf_counts(ta, tb, 7.5, 150)
        assert ho.sum() > 1000
        np.testing.assert_array_equal(hg, ho)


def test_zsampler_regimes_reached(jm):
    """Accepted MRZ jumps whose Z came from each regime of the sampler
    (eta < -1: Gamma(2) proposal; -1 <= eta <= 0: Rayleigh; eta > 0: mixed),
    as the oracle counts them, with the GPU's events and state identical."""
    sy, sp = water_small()
    pa = S.water_params()
    pa.log_events = 1
    g, o = _pair(jm, sy, sp, pa)
    g.step_jump(20)
    o.step_jump(20)
    reg = o.zsampler_regimes()
    assert (reg > 0).all(), reg
    np.testing.assert_array_equal(g.events(), o.events())
    xg, vg = g.state()
    xo, vo = o.state()
    assert rel_err(vg, vo) < TOL and rel_err(xg, xo) < TOL


def test_jump_water_100_steps(jm):
    """1001 waters (3003 atoms), the workload's split (5 / 10 A, 12 rings,
    skin 0.5 A) with automatic lanes and graph replays of 20 steps: 100 JUMP
    steps with every accepted jump identical, state within 1e-9."""
    sy = S.water_box(1001, seed=5, jitter=0.05)
    sp = S.water_split(r_s=5.0, r_c=10.0, w=1.0, skin=0.5, n_rings=12)
    pa = S.water_params(eps0_per_kcal=0.1)
    pa.log_events = 1
    pa.event_capacity = 1 << 24   # about 9.4M accepted jumps in 100 steps
    pa.graph_steps = 20
    g, o = _pair(jm, sy, sp, pa)
    g.step_jump(100)
    o.step_jump(100)
    xg, vg = g.state()
    xo, vo = o.state()
    assert rel_err(xg, xo) < TOL, rel_err(xg, xo)
    assert rel_err(vg, vo) < TOL, rel_err(vg, vo)
    sg, so = g.atom_stats(), o.atom_stats()
    for k in ("n_prop", "n_acc", "hash"):
        np.testing.assert_array_equal(sg[k], so[k], err_msg=k)
    eo = o.events()
    assert len(eo) > 100000
    np.testing.assert_array_equal(g.events(), eo)
    assert g.observables()["n_rebuilds"] == o.n_rebuilds
