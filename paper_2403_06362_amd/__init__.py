"""MI355X (gfx950) hash- vs stride-seeded LCG streams and slab Monte Carlo
transport: Python side of libmcrng.so (include/mcrng.h).

Paper: Cuneo & Variansyah, "An Alternative to Stride-Based RNG for Monte
Carlo Transport" (arXiv 2403.06362).

The entry points mirror the C ABI: init_streams, draw, uniforms, Context.run_histories,
Context.reduce_tallies, Context.run_pulse, Context.run_pulse_pc (plus Context.autotune), and
run_histories_noalloc (run and reduce without device allocation).  Tensors
are torch device tensors; the library does all the arithmetic.
`transport()`, `pulse()` and `pulse_pc()` are convenience wrappers that allocate the
output tensors.
"""
from ._binding import (  # noqa: F401
    DIAG_NAMES, EXPORTS, FP32, FP64, NDIAG, PULSE_AUTO, PULSE_BANK, PULSE_DIAG_NAMES, PULSE_EVENT, PULSE_FAMILY,
    SCHED_EVENT, SCHED_HISTORY, Context, McrngError, PulseOpts, PulsePc, RunOpts, draw, init_streams, lib,
    make_opts, make_pulse_opts, make_pulse_pc, pulse_n_census, run_histories_noalloc, tally_bins, uniforms,
)

__all__ = ["init_streams", "draw", "uniforms", "Context", "run_histories_noalloc", "RunOpts", "make_opts", "tally_bins", "transport", "pulse",
           "PulseOpts", "make_pulse_opts", "pulse_pc", "PulsePc", "make_pulse_pc", "pulse_n_census", "McrngError", "lib", "FP64", "FP32", "SCHED_HISTORY", "SCHED_EVENT",
           "PULSE_AUTO", "PULSE_BANK", "PULSE_FAMILY", "PULSE_EVENT", "NDIAG", "DIAG_NAMES", "PULSE_DIAG_NAMES"]


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


def pulse(problem, lcg, ctx=None, opts=None, stream=None, device="cuda:0"):
    """Runs a pulse problem.  Returns (counts, flux, diag): counts a uint64
    tensor [n_batches, n_time_bins], flux float64 of the same shape, diag a
    uint64 tensor [NDIAG]."""
    import torch
    own = ctx is None
    ctx = ctx or Context(torch.device(device).index or 0)
    try:
        nt = len(problem.time_edges) - 1
        counts = torch.empty((problem.n_batches, nt), dtype=torch.uint64, device=device)
        flux = torch.empty((problem.n_batches, nt), dtype=torch.float64, device=device)
        diag = torch.empty(NDIAG, dtype=torch.uint64, device=device)
        ctx.run_pulse(lcg, problem, counts, flux, diag, opts, stream)
        return counts, flux, diag
    finally:
        if own:
            torch.cuda.synchronize()
            ctx.close()


def pulse_pc(problem, lcg, ctx=None, opts=None, stream=None, device="cuda:0"):
    """Runs a pulse problem with population control (problem.census_every,
    pc_target, pc_seed; hash seeding).  Returns (counts, flux, diag, pop):
    pop a uint64 tensor [n_batches, n_census, 2] (arrivals, copies)."""
    import torch
    own = ctx is None
    ctx = ctx or Context(torch.device(device).index or 0)
    try:
        nt = len(problem.time_edges) - 1
        nc = pulse_n_census(problem)
        counts = torch.empty((problem.n_batches, nt), dtype=torch.uint64, device=device)
        flux = torch.empty((problem.n_batches, nt), dtype=torch.float64, device=device)
        diag = torch.empty(NDIAG, dtype=torch.uint64, device=device)
        pop = torch.empty((problem.n_batches, max(nc, 1), 2), dtype=torch.uint64, device=device)
        ctx.run_pulse_pc(lcg, problem, counts, flux, diag, pop if nc else None, opts, stream)
        return counts, flux, diag, pop[:, :nc]
    finally:
        if own:
            torch.cuda.synchronize()
            ctx.close()
