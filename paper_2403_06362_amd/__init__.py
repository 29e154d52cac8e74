"""MI355X (gfx950) hash- vs stride-seeded LCG streams and slab Monte Carlo
transport: Python side of libmcrng.so (include/mcrng.h).

Paper: Cuneo & Variansyah, "An Alternative to Stride-Based RNG for Monte
Carlo Transport" (arXiv 2403.06362).

The entry points mirror the C ABI: init_streams, draw, Context.run_histories,
Context.reduce_tallies (plus Context.autotune).  Tensors are torch device
tensors; the library does all the arithmetic.  `transport()` is a
convenience wrapper that allocates the output tensors.
"""
from ._binding import (  # noqa: F401
    DIAG_NAMES, EXPORTS, FP32, FP64, NDIAG, SCHED_EVENT, SCHED_HISTORY, Context, McrngError, RunOpts,
    draw, init_streams, lib, make_opts, tally_bins,
)

__all__ = ["init_streams", "draw", "Context", "RunOpts", "make_opts", "tally_bins", "transport",
           "McrngError", "lib", "FP64", "FP32", "SCHED_HISTORY", "SCHED_EVENT", "NDIAG", "DIAG_NAMES"]


def transport(problems, lcg, ctx=None, opts=None, stream=None, device="cuda:0"):
    """Runs the problems and reduces their tallies.  Returns (raw, flux,
    diag): raw is a uint64 tensor [bins, 2] (low, high words of the exact
    128-bit sums), flux a float64 tensor [bins], diag a uint64 tensor
    [n_problems, NDIAG]."""
    import torch
    own = ctx is None
    ctx = ctx or Context(torch.device(device).index or 0)
    try:
        nb = tally_bins(problems)
        raw = torch.empty((max(nb, 1), 2), dtype=torch.uint64, device=device)
        flux = torch.empty(max(nb, 1), dtype=torch.float64, device=device)
        diag = torch.empty((len(problems), NDIAG), dtype=torch.uint64, device=device)
        ctx.run_histories(lcg, problems, opts, stream)
        ctx.reduce_tallies(raw, flux, diag, stream)
        return raw[:nb], flux[:nb], diag
    finally:
        if own:
            torch.cuda.synchronize()
            ctx.close()
