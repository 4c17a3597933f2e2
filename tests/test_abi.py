"""The C ABI library loads and exports every function include/jumpmd.h declares
(no compute calls: runs without a GPU)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "jumpmd.h")
LIB = os.path.join(ROOT, "paper_2412_15073_amd", "libjumpmd.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(md_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    fns = declared_functions()
    for f in ("md_create", "md_step_baoab", "md_step_jump", "md_step_jump_respa", "md_observables",
              "md_destroy", "md_last_error"):
        assert f in fns


@pytest.mark.skipif(not os.path.exists(LIB), reason="libjumpmd.so not built")
def test_library_exports_every_declared_function():
    lib = C.CDLL(LIB)
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libjumpmd.so not built")
def test_binding_covers_every_export():
    from paper_2412_15073_amd import jumpmd
    assert sorted(jumpmd.EXPORTS) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libjumpmd.so not built")
def test_create_rejects_bad_arguments_without_touching_the_device():
    """Validation happens before any HIP call: bad splits fail with MD_ERR_ARG."""
    from paper_2412_15073_amd import jumpmd, systems as S
    sy = S.lj_fcc(4)
    bad = S.Split(r_s=2.0, r_c=6.5, switch_width=0.5, skin=0.3)   # r_c + skin above the box edge
    with pytest.raises(jumpmd.MDError) as e:
        jumpmd.Sim(sy, bad, S.lj_params(), stream=0)
    assert e.value.code == jumpmd.MD_ERR_ARG
    bad = S.Split(r_s=1.5, r_c=3.0, switch_width=0.5, skin=0.3)   # r_s - w below 1.25 sigma
    with pytest.raises(jumpmd.MDError) as e:
        jumpmd.Sim(sy, bad, S.lj_params(), stream=0)
    assert e.value.code == jumpmd.MD_ERR_ARG


@pytest.mark.skipif(not os.path.exists(LIB), reason="libjumpmd.so not built")
def test_theta_screen_check_rejects_bad_arguments_without_touching_the_device():
    from paper_2412_15073_amd import jumpmd
    for lo, hi, n in ((-5.0, 60.0, 1), (1.0, 1.0, 100), (2.0, -1.0, 100)):
        with pytest.raises(jumpmd.MDError) as e:
            jumpmd.theta_screen_error(lo, hi, n)
        assert e.value.code == jumpmd.MD_ERR_ARG


def _rejects(sy, sp, pa):
    from paper_2412_15073_amd import jumpmd
    with pytest.raises(jumpmd.MDError) as e:
        jumpmd.Sim(sy, sp, pa, stream=0)
    assert e.value.code == jumpmd.MD_ERR_ARG, e.value
    return str(e.value)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libjumpmd.so not built")
def test_create_rejects_bad_topology_without_touching_the_device():
    """Bond, angle and exclusion indices outside [0, N), terms spanning two
    replicas, non-monotone exclusion offsets and replicas of fewer than two
    atoms are refused with MD_ERR_ARG before any device work (they would
    otherwise index out of bounds on the host and the device)."""
    import numpy as np
    from paper_2412_15073_amd import systems as S
    sp = S.water_split(r_s=5.0, r_c=7.0, w=1.0, skin=0.5, n_rings=3)
    pa = S.water_params()
    base = S.water_box(125, seed=3)
    sy = S.with_(base, bond_ij=base.bond_ij.copy())
    sy.bond_ij[7, 1] = sy.n_atoms            # out of range
    assert "bond" in _rejects(sy, sp, pa)
    sy = S.with_(base, angle_ijk=base.angle_ijk.copy())
    sy.angle_ijk[3, 2] = -1
    assert "angle" in _rejects(sy, sp, pa)
    sy = S.with_(base, excl_j=base.excl_j.copy())
    sy.excl_j[5] = sy.n_atoms + 3
    assert "exclusion" in _rejects(sy, sp, pa)
    sy = S.with_(base, excl_ptr=base.excl_ptr.copy())
    sy.excl_ptr[10], sy.excl_ptr[11] = sy.excl_ptr[11], sy.excl_ptr[10]
    assert "excl_ptr" in _rejects(sy, sp, pa)
    # a bond across the two replicas of a batch
    a, b = S.water_box(125, seed=3), S.water_box(125, seed=4)
    a = S.with_(a, bond_ij=a.bond_ij.copy())
    a.bond_ij[0, 1] = a.n_atoms + 1          # global index into the second replica
    assert "replica" in _rejects(S.Batch([a, b]), sp, pa)
    # a replica of a single atom
    one = S.with_(b, n_atoms=1, pos=b.pos[:1], vel=b.vel[:1], mass=b.mass[:1], charge=b.charge[:1],
                  type=b.type[:1], bond_ij=np.zeros((0, 2), np.int32), bond_k=np.zeros(0), bond_r0=np.zeros(0),
                  angle_ijk=np.zeros((0, 3), np.int32), angle_k=np.zeros(0), angle_t0=np.zeros(0),
                  excl_ptr=np.zeros(2, np.int32), excl_j=np.zeros(0, np.int32))
    assert "replica_offset" in _rejects(S.Batch([S.water_box(125, seed=3), one]), sp, pa)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libjumpmd.so not built")
def test_create_rejects_bad_knobs_and_allocator():
    from paper_2412_15073_amd import jumpmd, systems as S
    sy = S.lj_fcc(4)
    sp = S.Split(r_s=2.0, r_c=3.0, switch_width=0.5, skin=0.3)
    pa = S.lj_params()
    pa.bound_scale = -1.0
    assert "bound_scale" in _rejects(sy, sp, pa)
    pa = S.lj_params()
    pa.row_capacity = float("nan")
    assert "row_capacity" in _rejects(sy, sp, pa)
    # an allocator without its release callback
    half = jumpmd.MDAllocator()
    half.alloc = jumpmd._ALLOC_FN(lambda c, n, s: None)

    class Half:
        struct = half
    with pytest.raises(jumpmd.MDError) as e:
        jumpmd.Sim(sy, sp, S.lj_params(), stream=0, allocator=Half())
    assert e.value.code == jumpmd.MD_ERR_ARG and "release" in str(e.value)
