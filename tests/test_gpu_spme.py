"""Smooth particle-mesh Ewald on the GPU (spreading, transforms, influence
function, gather) against the oracle's plain SPME: reciprocal-space forces
within 1e-12 for every B-spline order and a non-cubic grid (the four-launch
path), and for meshes with large (y, z) planes (the other two spreading
paths), energies within
1e-9, JUMP-RESPA1 and plain JUMP runs with identical jump events and FP64
state within 1e-9, and the 4096-water box at the paper's 12 000-atom
settings (alpha 0.554, 64^3 grid). Spreading sums with atomics, so two GPU
runs agree to rounding only; the tolerances hold for either order."""
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


def _spme_water(n_mol=125, seed=31, alpha=0.3, grid=(16, 32, 16), order=6, r_c=7.0):
    sy = S.water_box(n_mol, seed=seed, jitter=0.05)
    sp = S.water_split(r_s=5.0, r_c=r_c, w=1.0, skin=0.5, alpha=alpha, n_rings=3)
    sp.coulomb_kind, sp.pme_grid, sp.pme_order = S.COUL_SPME, grid, order
    return sy, sp


@pytest.mark.parametrize("order", [4, 6, 8])
def test_spme_forces(jm, order):
    from oracle.oracle import OracleSim, F_RECIP
    sy, sp = _spme_water(order=order)
    g, o = jm.Sim(sy, sp, S.water_params()), OracleSim(sy, sp, S.water_params())
    fo = o.accel(F_RECIP)
    assert np.abs(fo).max() > 0.0
    assert rel_err(g.accel(4), fo) < 1e-12


@pytest.mark.parametrize("grid", [(8, 64, 128), (8, 128, 128), (256, 8, 16)])
def test_spme_forces_other_paths(jm, grid):
    """Meshes whose (y, z) plane does not fit LDS as complex FP64: spreading by
    real planes in LDS (K1 K2 = 8192), and by global atomics (16384), each with
    the six axis passes; and a 256-point first axis on the four-launch path
    (8 x lines per block). Forces and energy against the oracle."""
    from oracle.oracle import OracleSim, F_RECIP
    sy, sp = _spme_water(seed=36, grid=grid, order=4)
    g, o = jm.Sim(sy, sp, S.water_params(jumps=False)), OracleSim(sy, sp, S.water_params(jumps=False))
    assert rel_err(g.accel(4), o.accel(F_RECIP)) < 1e-12
    eg, eo = g.observables(pe=True)["pe_recip"], o.energies()["pe_recip"]
    assert abs(eg - eo) <= TOL * abs(eo), (eg, eo)


def test_spme_energy(jm):
    from oracle.oracle import OracleSim
    sy, sp = _spme_water(seed=32)
    g, o = jm.Sim(sy, sp, S.water_params(jumps=False)), OracleSim(sy, sp, S.water_params(jumps=False))
    g.step_baoab(5)
    o.step_baoab(5)
    eg, eo = g.observables(pe=True)["pe_recip"], o.energies()["pe_recip"]
    assert abs(eg - eo) <= TOL * abs(eo), (eg, eo)


@pytest.mark.parametrize("scheme", ["jump_respa1", "jump"])
def test_spme_jump_trajectories(jm, scheme):
    """JUMP-RESPA1 at 1:2:6 fs (4 outer steps) and plain JUMP (12 steps)
    with SPME reciprocal forces: identical events and state."""
    from oracle.oracle import OracleSim
    sy, sp = _spme_water(seed=33)
    pa = S.water_params()
    pa.respa_inner, pa.respa_outer = 2, 3
    pa.log_events = 1
    g, o = jm.Sim(sy, sp, pa), OracleSim(sy, sp, pa)
    n = 4 if scheme == "jump_respa1" else 12
    getattr(g, "step_" + scheme)(n)
    getattr(o, "step_" + scheme)(n)
    xg, vg = g.state()
    xo, vo = o.state()
    assert rel_err(xg, xo) < TOL and rel_err(vg, vo) < TOL
    sg, so = g.atom_stats(), o.atom_stats()
    for k in ("n_prop", "n_acc", "hash"):
        np.testing.assert_array_equal(sg[k], so[k], err_msg=k)
    ev = o.events()
    assert len(ev) > 1000
    np.testing.assert_array_equal(g.events(), ev)


def test_spme_baoab_respa1_trajectory(jm):
    from oracle.oracle import OracleSim
    sy, sp = _spme_water(seed=34, order=4)
    pa = S.water_params(jumps=False)
    pa.respa_inner, pa.respa_outer = 2, 2
    g, o = jm.Sim(sy, sp, pa), OracleSim(sy, sp, pa)
    g.step_baoab_respa1(6)
    o.step_baoab_respa1(6)
    xg, vg = g.state()
    xo, vo = o.state()
    assert rel_err(xg, xo) < TOL and rel_err(vg, vo) < TOL


def test_spme_full_size_paper_settings(jm):
    """The 4096-water box (49.7 A) with the paper's Ewald settings for its
    12 000-atom system: alpha 0.554, real space to 7 A, a 64^3 grid (the
    paper's is 60^3), order 6: reciprocal forces within 1e-12 of the
    oracle, and within 2e-3 of the plain Ewald sum at |n| <= 34 (the mesh's
    own interpolation error: 6e-4 relative to the largest force)."""
    from oracle.oracle import OracleSim, F_RECIP
    sy = S.water_box(4096, seed=1)
    sp = S.water_split(r_s=5.0, r_c=7.0, w=0.5, skin=0.5, alpha=0.554, n_rings=6)
    sp.coulomb_kind, sp.pme_grid, sp.pme_order = S.COUL_SPME, (64, 64, 64), 6
    g = jm.Sim(sy, sp, S.water_params())
    fg = g.accel(4)
    fo = OracleSim(sy, sp, S.water_params()).accel(F_RECIP)
    assert rel_err(fg, fo) < 1e-12
    sp.coulomb_kind, sp.ewald_kmax = S.COUL_EWALD, 34
    fe = jm.Sim(sy, sp, S.water_params()).accel(4)
    assert rel_err(fg, fe) < 2e-3


def test_spme_rejects_bad_grids(jm):
    sy, sp = _spme_water(seed=35)
    for grid, order in (((12, 16, 16), 6), ((16, 16, 16), 5), ((4, 16, 16), 6), ((16, 16, 512), 6)):
        sp.pme_grid, sp.pme_order = grid, order
        with pytest.raises(jm.MDError) as e:
            jm.Sim(sy, sp, S.water_params())
        assert e.value.code == jm.MD_ERR_ARG
