"""Velocity trace (md_trace_velocities / md_get_trace): one record per O
update, i.e. per smallest time step, for the autocorrelation spectra of
Sec. 4 (Figs. 3-4 are taken at the level of the smallest step). The
records are the mid-step velocities of BAOAB (checked against the end-of-step
state and forces), their count and order follow the steps of every scheme,
the ring keeps the last records, and tracing leaves the trajectory unchanged
(it only turns HIP-graph replay off)."""
import numpy as np
import pytest

from paper_2412_15073_amd import systems as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def jm():
    from paper_2412_15073_amd import jumpmd
    jumpmd.load()
    return jumpmd


def _water(n_mol=125, seed=21):
    sy = S.water_box(n_mol, seed=seed, jitter=0.05)
    sp = S.water_split(r_s=5.0, r_c=7.0, w=1.0, skin=0.5, n_rings=3)
    return sy, sp


def _ewald(n_mol=125, seed=22):
    sy = S.water_box(n_mol, seed=seed, jitter=0.05)
    sp = S.water_split(r_s=5.0, r_c=7.0, w=1.0, skin=0.5, alpha=0.3, n_rings=3)
    sp.coulomb_kind, sp.ewald_kmax = S.COUL_EWALD, 8
    return sy, sp


@pytest.mark.parametrize("graph", [0, 4])
def test_baoab_records_are_the_mid_step_velocities(jm, graph):
    """BAOAB: B A O A B, so the velocity after O is v_end - (dt/2) a(x_end)
    with the full non-bonded plus bonded acceleration at the end positions."""
    sy, sp = _water()
    pa = S.water_params(jumps=False)
    pa.graph_steps = graph
    g = jm.Sim(sy, sp, pa)
    n = 40
    g.trace_velocities(sy.n_atoms, 64)
    want = []
    for _ in range(n):
        g.step_baoab(1)
        _, v = g.state()
        a = g.accel(1) + g.accel(2)
        want.append(v - 0.5 * pa.dt * a)
    rec, tn = g.trace()
    assert tn == n and rec.shape == (n, sy.n_atoms, 3)
    want = np.array(want)
    assert np.abs(rec - want).max() < 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("scheme,m,p", [("baoab", 1, 1), ("jump", 1, 1), ("jump_respa", 3, 1),
                                        ("jump_respa1", 2, 3), ("baoab_respa1", 2, 3)])
def test_trace_counts_and_unchanged_trajectory(jm, scheme, m, p):
    """One record per inner step (m p per call of a RESPA1 step, m per
    RESPA step), and the same final state with and without tracing (graphs
    of 4 steps where the scheme replays them)."""
    ew = scheme.endswith("respa1")
    sy, sp = _ewald() if ew else _water()
    pa = S.water_params(jumps=scheme.startswith("jump"))
    pa.graph_steps = 4
    pa.respa_inner = m
    pa.respa_outer = p
    n_atoms = 30
    out = []
    for traced in (False, True):
        g = jm.Sim(sy, sp, pa)
        if traced:
            g.trace_velocities(n_atoms, 1000)
        getattr(g, "step_" + scheme)(8)
        out.append(g.state())
        if traced:
            rec, tn = g.trace()
            assert tn == 8 * m * p and rec.shape == (8 * m * p, n_atoms, 3)
            assert np.isfinite(rec).all() and np.abs(rec).max() > 0.0
    (x0, v0), (x1, v1) = out
    assert np.abs(x1 - x0).max() <= 1e-14 * np.abs(x0).max()
    assert np.abs(v1 - v0).max() <= 1e-14 * np.abs(v0).max()


@pytest.mark.parametrize("scheme", ["baoab_respa", "baoab_respa1"])
def test_respa_records_are_the_last_inner_step_velocities(jm, scheme):
    """The record of the last inner step of an outer step is the velocity
    after its O update: the end-of-step velocity minus the kicks that follow
    it (inner bonded half kick; BAOAB-RESPA: the full non-bonded outer half
    kick; BAOAB-RESPA1: the short middle half kick and the reciprocal plus
    long real-space outer half kick), all at the end positions. Every record
    is a different inner step (the O noise makes consecutive records differ)."""
    ew = scheme.endswith("respa1")
    sy, sp = _ewald(seed=25) if ew else _water(seed=25)
    pa = S.water_params(jumps=False)
    m, p = (2, 3) if ew else (3, 1)
    pa.respa_inner, pa.respa_outer = m, p
    g = jm.Sim(sy, sp, pa)
    g.trace_velocities(sy.n_atoms, 4 * m * p)
    h = 0.5 * pa.dt
    for call in range(4):
        getattr(g, "step_" + scheme)(1)
        _, v = g.state()
        if ew:
            want = v - h * g.accel(2) - m * h * g.accel(0) - p * m * h * (g.accel(4) + g.accel(3))
        else:
            want = v - h * g.accel(2) - m * h * g.accel(1)
        rec, tn = g.trace()
        assert tn == (call + 1) * m * p
        assert np.abs(rec[-1] - want).max() < 1e-12 * np.abs(want).max()
    flat = rec.reshape(len(rec), -1)
    assert len(rec) == 4 * m * p
    assert all(np.abs(flat[k] - flat[k + 1]).max() > 0.0 for k in range(len(rec) - 1))


def test_ring_keeps_the_last_records(jm):
    sy, sp = _water(seed=23)
    pa = S.water_params(jumps=False)
    recs = []
    for cap in (100, 7):
        g = jm.Sim(sy, sp, pa)
        g.trace_velocities(12, cap)
        g.step_baoab(19)
        rec, tn = g.trace()
        assert tn == 19 and len(rec) == min(19, cap)
        recs.append(rec)
    assert np.array_equal(recs[0][-7:], recs[1])
    g.trace_velocities(0, 0)   # stops; a new trace counts from zero
    g.trace_velocities(12, 4)
    g.step_baoab(2)
    assert g.trace()[1] == 2


def test_trace_rejects_bad_arguments(jm):
    sy, sp = _water(seed=24)
    g = jm.Sim(sy, sp, S.water_params(jumps=False))
    for n_atoms, cap in ((-1, 10), (sy.n_atoms + 1, 10), (5, 0)):
        with pytest.raises(jm.MDError) as e:
            g.trace_velocities(n_atoms, cap)
        assert e.value.code == jm.MD_ERR_ARG
    g._trace = (1, 1)
    with pytest.raises(jm.MDError) as e:
        g.trace()   # no active trace
    assert e.value.code == jm.MD_ERR_ARG
