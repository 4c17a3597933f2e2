"""md_rdf_noalloc (the entry point for callers that cannot allocate device
memory) against md_rdf: identical counts on two calls in a row, the second on
a smaller system with fewer bins, with no device memory drawn meanwhile."""
import ctypes as C

import numpy as np
import pytest

from paper_2412_15073_amd import systems as S

pytestmark = pytest.mark.gpu

MAX_BINS = 16384


@pytest.fixture(scope="module")
def jm():
    from paper_2412_15073_amd import jumpmd
    jumpmd.load()
    return jumpmd


def _noalloc(jm, sim, ta, tb, r_max, n_bins):
    h = np.full(n_bins, -1.0)
    rc = jm.load().md_rdf_noalloc(sim._h, ta, tb, r_max, n_bins, h.ctypes.data_as(C.POINTER(C.c_double)))
    return rc, h


def test_noalloc_rdf_matches_rdf_twice_without_allocating(jm):
    import torch
    sp = S.water_split(r_s=5.0, r_c=7.0, w=1.0, skin=0.5, n_rings=3)
    pa = S.water_params()
    big = jm.Sim(S.water_box(343, seed=21, jitter=0.05), sp, pa)
    small = jm.Sim(S.water_box(125, seed=22, jitter=0.05), sp, pa)
    big.step_jump(20)
    small.step_jump(20)
    ref1 = big.rdf_counts(0, 0, 10.0, 400)        # O-O, allocating path
    ref2 = small.rdf_counts(0, 1, 6.0, 60)        # O-H, fewer bins, smaller system
    assert ref1.sum() > 1000 and ref2.sum() > 100
    torch.cuda.synchronize()
    mem0 = torch.cuda.memory_allocated()
    drawn0 = (big.allocator.bytes_total, small.allocator.bytes_total)
    rc, h1 = _noalloc(jm, big, 0, 0, 10.0, 400)
    assert rc == jm.MD_OK, jm.load().md_last_error(big._h)
    np.testing.assert_array_equal(h1, ref1)
    # second call: smaller input; the shared scratch still holds the first call's counts
    rc, h2 = _noalloc(jm, small, 0, 1, 6.0, 60)
    assert rc == jm.MD_OK, jm.load().md_last_error(small._h)
    np.testing.assert_array_equal(h2, ref2)
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == mem0
    assert (big.allocator.bytes_total, small.allocator.bytes_total) == drawn0
    # the stepping state is untouched: md_rdf after more steps still agrees
    big.step_jump(5)
    rc, h3 = _noalloc(jm, big, 1, 1, 8.0, MAX_BINS)
    assert rc == jm.MD_OK
    np.testing.assert_array_equal(h3, big.rdf_counts(1, 1, 8.0, MAX_BINS))
    # beyond the static scratch: a clear error, nothing written
    rc, h4 = _noalloc(jm, big, 0, 0, 10.0, MAX_BINS + 1)
    assert rc == jm.MD_ERR_ARG
    assert b"static scratch" in jm.load().md_last_error(big._h)
    assert np.all(h4 == -1.0)
    big.close()
    small.close()
