"""The autotuner (md_tune): it times settings that leave the method's law
unchanged and returns the fastest; the choice is one of the timed settings,
the minimum of them, valid for md_create, and cached per process."""
import time

import numpy as np
import pytest

from paper_2412_15073_amd import systems as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def jm():
    from paper_2412_15073_amd import jumpmd
    jumpmd.load()
    return jumpmd


@pytest.mark.parametrize("scheme", ["jump", "baoab"])
def test_tuner_returns_the_fastest_timed_setting(jm, scheme):
    sy = S.water_box(343, seed=51, jitter=0.05)
    sp = S.water_split(r_s=5.0, r_c=7.0, w=1.0, skin=0.5, n_rings=4)
    pa = S.water_params(jumps=(scheme == "jump"))
    sp2, pa2, ms, trials = jm.tune(sy, sp, pa, scheme=scheme, steps=20)
    assert len(trials) >= (10 if scheme == "jump" else 5)
    assert ms > 0 and ms == min(t["ms_per_step"] for t in trials)
    best = [t for t in trials if t["ms_per_step"] == ms][0]
    assert (best["chain_lanes"], best["skin"], best["n_rings"], best["graph_steps"]) == \
        (pa2.chain_lanes, sp2.skin, sp2.n_rings, pa2.graph_steps)
    assert sp2.r_s == sp.r_s and sp2.r_c == sp.r_c and pa2.dt == pa.dt and pa2.eps == pa.eps
    if sp2.n_rings > 1:   # rings span the candidate distances
        span = (sp2.r_c + sp2.skin) - (sp2.r_s - sp2.switch_width - sp2.skin)
        assert abs(sp2.ring_width * sp2.n_rings - span) < 1e-12
    if scheme == "baoab":
        assert all(t["chain_lanes"] == pa.chain_lanes for t in trials)
    # cached: the same answer at once, no trials run
    t0 = time.perf_counter()
    sp3, pa3, ms3, trials3 = jm.tune(sy, sp, pa, scheme=scheme, steps=20)
    assert time.perf_counter() - t0 < 0.5
    assert ms3 == ms and len(trials3) == len(trials) and sp3.skin == sp2.skin and pa3.chain_lanes == pa2.chain_lanes
    # the chosen setting runs
    g = jm.Sim(sy, sp2, pa2)
    (g.step_jump if scheme == "jump" else g.step_baoab)(20)
    assert np.isfinite(g.observables()["temperature"])


def test_tuned_lanes_do_not_change_results(jm):
    """Lanes per atom are a pure launch setting: the tuned choice gives the
    same trajectory and jump fingerprints as one lane per atom."""
    sy = S.water_box(216, seed=52, jitter=0.05)
    sp = S.water_split(r_s=5.0, r_c=7.0, w=1.0, skin=0.5, n_rings=4)
    pa = S.water_params()
    sp2, pa2, _, _ = jm.tune(sy, sp, pa, scheme="jump", steps=20)
    pa1 = S.water_params()
    pa1.chain_lanes = 1
    pa1.graph_steps = 0
    g1, g2 = jm.Sim(sy, sp2, pa1), jm.Sim(sy, sp2, pa2)
    g1.step_jump(10)
    g2.step_jump(10)
    x1, v1 = g1.state()
    x2, v2 = g2.state()
    np.testing.assert_array_equal(g1.atom_stats()["hash"], g2.atom_stats()["hash"])
    assert np.abs(x1 - x2).max() < 1e-9 * np.abs(x1).max()
    assert np.abs(v1 - v2).max() < 1e-9 * np.abs(v1).max()


def test_tuner_rejects_bad_arguments(jm):
    sy = S.water_box(125, seed=53)
    sp = S.water_split(r_s=5.0, r_c=7.0, w=1.0, skin=0.5, n_rings=4)
    with pytest.raises(jm.MDError) as e:
        jm.tune(sy, sp, S.water_params(), scheme="jump", steps=0)
    assert e.value.code == jm.MD_ERR_ARG


@pytest.mark.parametrize("lanes", [1, 2])
def test_chain_wave_order_does_not_change_results(jm, lanes):
    """The wave order of the jump chains (by type, or replica by replica) is a
    pure launch setting: identical fingerprints and state on a batch."""
    reps = [S.water_box(m, seed=60 + k, jitter=0.05) for k, m in enumerate((216, 250, 300, 340))]
    sp = S.water_split(r_s=5.0, r_c=7.0, w=1.0, skin=0.5, n_rings=4)
    out = []
    for order in (1, 2):
        pa = S.water_params()
        pa.chain_lanes, pa.chain_order = lanes, order
        g = jm.Sim(S.Batch(reps), sp, pa)
        g.step_jump(8)
        out.append((g.state(), g.atom_stats()))
    (x1, v1), s1 = out[0]
    (x2, v2), s2 = out[1]
    for k in ("n_prop", "n_acc", "hash"):
        np.testing.assert_array_equal(s1[k], s2[k], err_msg=k)
    assert np.abs(x1 - x2).max() < 1e-9 * np.abs(x1).max()
    assert np.abs(v1 - v2).max() < 1e-9 * np.abs(v1).max()
