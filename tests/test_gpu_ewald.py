"""Ewald electrostatics and the three-level RESPA schemes on the GPU against
the oracle: reciprocal-space forces (plain Ewald sum over the half space of
k-vectors, excluded-pair correction) and the long real-space part within
1e-12, energies within 1e-9, and BAOAB, JUMP-RESPA1 (1:2:6 fs, Sec. 2.3.2,
Table 2), BAOAB-RESPA1 and plain JUMP (reciprocal forces in the C'
acceleration) runs with identical jump events and FP64 state within 1e-9."""
import numpy as np
import pytest

from paper_2412_15073_amd import systems as S
from tests.helpers import rel_err

pytestmark = pytest.mark.gpu

TOL = 1e-9


@pytest.fixture(scope="module")
def jm():
    from paper_2412_15073_amd import jumpmd
    jumpmd.load()
    return jumpmd


def _ewald_water(n_mol=125, seed=9, alpha=0.3, kmax=8, r_c=7.0):
    sy = S.water_box(n_mol, seed=seed, jitter=0.05)
    sp = S.water_split(r_s=5.0, r_c=r_c, w=1.0, skin=0.5, alpha=alpha, n_rings=3)
    sp.coulomb_kind, sp.ewald_kmax = 1, kmax
    return sy, sp


def _pair(jm, sy, sp, pa):
    from oracle.oracle import OracleSim
    return jm.Sim(sy, sp, pa), OracleSim(sy, sp, pa)


def test_reciprocal_and_long_forces(jm):
    from oracle.oracle import F_RECIP, F_LONG
    sy, sp = _ewald_water()
    g, o = _pair(jm, sy, sp, S.water_params())
    fr = o.accel(F_RECIP)
    assert np.abs(fr).max() > 0.0
    assert rel_err(g.accel(4), fr) < 1e-12
    assert rel_err(g.accel(3), o.accel(F_LONG)) < 1e-12


def test_ewald_energies(jm):
    sy, sp = _ewald_water(seed=10)
    g, o = _pair(jm, sy, sp, S.water_params(jumps=False))
    g.step_baoab(5)
    o.step_baoab(5)
    og, oo = g.observables(pe=True), o.energies()
    for kg, ko in (("pe_recip", "pe_recip"), ("pe_short", "pe_short"), ("pe_long", "pe_long")):
        assert abs(og[kg] - oo[ko]) <= TOL * abs(oo[ko]), (kg, og[kg], oo[ko])


@pytest.mark.parametrize("graph", [0, 4])
def test_ewald_baoab_trajectory(jm, graph):
    sy, sp = _ewald_water(seed=11)
    pa = S.water_params(jumps=False)
    pa.graph_steps = graph
    g, o = _pair(jm, sy, sp, pa)
    g.step_baoab(20)
    o.step_baoab(20)
    xg, vg = g.state()
    xo, vo = o.state()
    assert rel_err(xg, xo) < TOL and rel_err(vg, vo) < TOL


@pytest.mark.parametrize("lanes", [2, 8])
def test_jump_respa1_trajectory(jm, lanes):
    """JUMP-RESPA1 at 1:2:6 fs (bonded 1 fs; short forces and jumps 2 fs;
    reciprocal forces 6 fs), 4 outer steps: identical events and state."""
    sy, sp = _ewald_water(seed=12)
    pa = S.water_params()
    pa.respa_inner, pa.respa_outer = 2, 3
    pa.log_events = 1
    pa.chain_lanes = lanes
    g, o = _pair(jm, sy, sp, pa)
    g.step_jump_respa1(4)
    o.step_jump_respa1(4)
    xg, vg = g.state()
    xo, vo = o.state()
    assert rel_err(xg, xo) < TOL and rel_err(vg, vo) < TOL
    sg, so = g.atom_stats(), o.atom_stats()
    for k in ("n_prop", "n_acc", "hash"):
        np.testing.assert_array_equal(sg[k], so[k], err_msg=k)
    ev = o.events()
    assert len(ev) > 1000
    np.testing.assert_array_equal(g.events(), ev)


def test_baoab_respa1_trajectory(jm):
    """BAOAB-RESPA1 at 1:2:4 fs, 5 outer steps, then 3 more: state within 1e-9."""
    sy, sp = _ewald_water(seed=13)
    pa = S.water_params(jumps=False)
    pa.respa_inner, pa.respa_outer = 2, 2
    g, o = _pair(jm, sy, sp, pa)
    g.step_baoab_respa1(5)
    g.step_baoab_respa1(3)
    o.step_baoab_respa1(8)
    xg, vg = g.state()
    xo, vo = o.state()
    assert rel_err(xg, xo) < TOL and rel_err(vg, vo) < TOL


@pytest.mark.parametrize("lanes,graph", [(2, 0), (8, 4)])
def test_jump_with_ewald_trajectory(jm, lanes, graph):
    """Plain JUMP with Ewald electrostatics: MRZ jumps of the damped
    real-space long part, the C' acceleration with the reciprocal-space
    forces re-evaluated every step; 12 steps (in HIP-graph chunks of 4 where
    set) with identical events and FP64 state within 1e-9."""
    sy, sp = _ewald_water(seed=15)
    pa = S.water_params()
    pa.log_events = 1
    pa.chain_lanes = lanes
    pa.graph_steps = graph
    g, o = _pair(jm, sy, sp, pa)
    g.step_jump(12)
    o.step_jump(12)
    xg, vg = g.state()
    xo, vo = o.state()
    assert rel_err(xg, xo) < TOL and rel_err(vg, vo) < TOL
    sg, so = g.atom_stats(), o.atom_stats()
    for k in ("n_prop", "n_acc", "hash"):
        np.testing.assert_array_equal(sg[k], so[k], err_msg=k)
    ev = o.events()
    assert len(ev) > 1000
    np.testing.assert_array_equal(g.events(), ev)


def test_ewald_refuses_other_schemes(jm):
    sy, sp = _ewald_water(seed=14)
    g = jm.Sim(sy, sp, S.water_params())
    for fn in (g.step_jump_respa, g.step_baoab_respa):
        with pytest.raises(jm.MDError) as e:
            fn(1)
        assert e.value.code == jm.MD_ERR_ARG
