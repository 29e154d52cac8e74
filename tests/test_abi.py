"""The C-ABI library loads and exports every symbol include/mcrng.h
declares; host-side validation rejects bad arguments before touching a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mcrng.h")


@pytest.fixture(scope="module")
def M():
    import paper_2403_06362_amd as M
    try:
        M.lib()
    except ImportError:
        pytest.fail("libmcrng.so is not built (run __graft_entry__.build())")
    return M


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mcrng_[a-z_0-9]+)\s*\(", text)))


def test_exports_every_declared_symbol(M):
    syms = declared_symbols()
    assert len(syms) >= 11
    assert sorted(M.EXPORTS) == syms
    lib = M.lib()
    for s in syms:
        assert hasattr(lib, s), s
    assert lib.mcrng_version() == 1


def test_host_validation_without_gpu(M):
    import workloads as W
    from paper_2403_06362_amd import _binding as B
    lib = M.lib()
    L = B.make_lcg(W.Lcg())
    S = B.make_seeding(W.hash_seeding())
    # NULL generator / seeding / buffers are rejected before any device work
    assert lib.mcrng_init_streams(None, C.byref(S), 10, None, None) == B.EINVAL
    assert "lcg" in lib.mcrng_last_error().decode()
    bad = B.Lcg(1, 1, 65, 0)
    assert lib.mcrng_init_streams(C.byref(bad), C.byref(S), 10, C.c_void_p(16), None) == B.EINVAL
    assert lib.mcrng_init_streams(C.byref(L), C.byref(S), 10, None, None) == B.EINVAL
    assert lib.mcrng_init_streams(C.byref(L), C.byref(S), 0, None, None) == B.OK   # n = 0: no-op
    assert lib.mcrng_draw(C.byref(L), None, 10, C.c_void_p(16), None, C.c_void_p(16), None) == B.EINVAL
    stride0 = B.Seeding(0, 0, 1, 0, 0, 0)
    assert lib.mcrng_init_streams(C.byref(L), C.byref(stride0), 4, C.c_void_p(16), None) == B.EINVAL
    assert lib.mcrng_run_histories(None, C.byref(L), None, 1, None, None) == B.EINVAL
    assert lib.mcrng_reduce_tallies(None, None, None, None, None) == B.EINVAL


def test_tally_bins_host_only(M):
    import workloads as W
    probs = [W.small_slab(), W.long_chain(n_histories=10), W.multi_region(n_histories=10)]
    assert M.tally_bins(probs) == 20 + 64 * 200 + 20 * 50
