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
    return sorted(set(re.findall(r"\b(md_[a-z_]+)\s*\(", text)))


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
    bad = S.Split(r_s=2.0, r_c=3.5, switch_width=0.5, skin=0.3)   # r_c above half the box
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
