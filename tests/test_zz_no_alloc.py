"""The allocation-free entry point (mcrng_run_histories_noalloc) against the
context-based run (mcrng_run_histories + mcrng_reduce_tallies) with the
same options: raw sums, flux and diagnostics bit for bit, on two calls in a
row (the second smaller, so that the static scratch still holds the first
call's larger contents), and a run too large for the scratch is rejected
without disturbing the next call."""
import sys

import numpy as np
import pytest

import workloads as W
from helpers import diag_dict, raw_ints

pytestmark = pytest.mark.gpu
LCG = W.Lcg()


def say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def M():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2403_06362_amd as M
    M.lib()
    return M


def _outputs(M, probs):
    import torch
    nb = M.tally_bins(probs)
    raw = torch.empty((nb, 2), dtype=torch.uint64, device="cuda:0")
    flux = torch.empty(nb, dtype=torch.float64, device="cuda:0")
    diag = torch.empty((len(probs), M.NDIAG), dtype=torch.uint64, device="cuda:0")
    return raw, flux, diag


def _noalloc(M, probs, **opts):
    import torch
    raw, flux, diag = _outputs(M, probs)
    raw.view(torch.int64).fill_(0xAB)
    flux.fill_(-1.0)
    M.run_histories_noalloc(LCG, probs, raw, flux, diag, opts=M.make_opts(**opts))
    torch.cuda.synchronize()
    return raw_ints(raw), flux.cpu().numpy(), diag_dict(diag, M.DIAG_NAMES)


def _with_context(M, probs, **opts):
    import torch
    ctx = M.Context(0)
    try:
        raw, flux, diag = M.transport(probs, LCG, ctx=ctx, opts=M.make_opts(**opts))
        torch.cuda.synchronize()
        return raw_ints(raw), flux.cpu().numpy(), diag_dict(diag, M.DIAG_NAMES)
    finally:
        ctx.close()


def test_noalloc_equals_context_run_twice(M):
    big = (W.batched(seeding_kind="stride", scale=2e-3)[:40] + [W.multi_region(n_histories=50_003)] +
           W.batched(scale=1e-3)[40:60])
    small = [W.small_slab(W.hash_seeding(), n_histories=3001)]
    chained = [W.long_chain(n_histories=2_000_003, n_batches=4)]   # units of 5200: the chained kernel
    cases = ((big, {}), (small, dict(block=128, hist_per_lane=2, precision=1)),
             (big[:7], dict(unit_histories=700, tally_copies=2)), (chained, dict(unit_histories=5200)))
    for i, (probs, opts) in enumerate(cases):
        say("noalloc call", i, len(probs), opts)
        got = _noalloc(M, probs, **opts)
        want = _with_context(M, probs, **opts)
        assert got[0] == want[0], i
        assert np.array_equal(got[1], want[1]), i
        assert got[2] == want[2], i


def test_noalloc_rejects_a_run_beyond_the_scratch(M):
    import torch
    huge = [W.homogeneous(40.0, 1.0, 0.9, 4000, 1_000_000)]   # 1954 units x 4000 bins x 16 B
    raw, flux, diag = _outputs(M, huge)
    say("noalloc too large")
    with pytest.raises(M.McrngError) as e:
        M.run_histories_noalloc(LCG, huge, raw, flux, diag, opts=M.make_opts(unit_histories=512))
    assert e.value.code == -1 and "static scratch" in str(e.value)
    torch.cuda.synchronize()
    probs = [W.small_slab(W.stride_seeding(), n_histories=2000)]
    say("noalloc after the rejection")
    got = _noalloc(M, probs)
    want = _with_context(M, probs)
    assert got[0] == want[0] and got[2] == want[2]
    assert np.array_equal(got[1], want[1])
