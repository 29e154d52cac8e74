"""GPU parity of the population-controlled pulse problem
(mcrng_run_pulse_pc) against the CPU oracle.

Population control at census times uses one-off hashed values of a
per-phase seed with each arrival's own state as the key, and seeds the
copies by eq. (5).  So the result does not depend on the order in which
the GPU banks its arrivals.  The bar is bit-exact counts, census
populations, flux and diagnostics, for every launch shape, including runs
that go through several chunks of batches."""
import sys

import numpy as np
import pytest

import workloads as W
from helpers import u64_np

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


@pytest.fixture(scope="module")
def ctx(M):
    c = M.Context(0)
    yield c
    c.close()


def run(M, ctx, prob, **opts):
    import torch
    counts, flux, diag, pop = M.pulse_pc(prob, LCG, ctx=ctx, opts=M.make_pulse_opts(**opts))
    torch.cuda.synchronize()
    d = dict(zip(M.PULSE_DIAG_NAMES, (int(v) for v in u64_np(diag))))
    nc = M.pulse_n_census(prob)
    return (u64_np(counts).reshape(prob.n_batches, -1), flux.cpu().numpy(), d,
            u64_np(pop.contiguous()).reshape(prob.n_batches, nc, 2))


def check(orc, prob, counts, flux, diag, pop, threads=8):
    ref = orc.pulse_pc(prob, LCG, threads=threads)
    assert np.array_equal(pop, ref.pop)
    assert np.array_equal(counts, ref.counts)
    assert diag == ref.diag
    assert np.array_equal(flux, orc.pulse_pc_flux(prob, LCG, ref.counts, ref.pop))
    return ref


def test_small_pc_parity(M, ctx, orc):
    p = W.pulse_pc(n_batches=10, per_batch=100, census_every=5)
    say("small pc")
    check(orc, p, *run(M, ctx, p))


def test_shapes_bit_identical(M, ctx, orc):
    p = W.pulse_pc(n_batches=13, per_batch=257, census_every=3, target=300).with_(first_batch=9)
    ref = orc.pulse_pc(p, LCG, threads=8)
    for block, chunk in ((64, 0), (128, 64), (256, 0), (256, 3000), (512, 0), (1024, 0)):
        say("pc shape", block, chunk)
        c, f, d, pop = run(M, ctx, p, block=block, schedule=M.PULSE_BANK, chunk=chunk)
        assert np.array_equal(pop, ref.pop), block
        assert np.array_equal(c, ref.counts), block
        assert d == ref.diag


def test_finish_launches_bit_identical(M, ctx, orc):
    """Census arrivals banked by finish launches (depth first per lane) are
    the same arrivals: every switch point gives the same populations."""
    p = W.pulse_pc(n_batches=6, per_batch=500, census_every=4, target=700)
    ref = orc.pulse_pc(p, LCG, threads=6)
    for div in (0xFFFFFFFF, 1, 3, 16):
        say("pc finish_div", div)
        c, _, d, pop = run(M, ctx, p, finish_div=div)
        assert np.array_equal(pop, ref.pop), div
        assert np.array_equal(c, ref.counts), div
        assert d == ref.diag, div


def test_event_schedule_with_population_control(M, ctx, orc):
    p = W.pulse_pc(n_batches=7, per_batch=300, census_every=3, target=250)
    ref = orc.pulse_pc(p, LCG, threads=7)
    for div in (0xFFFFFFFF, 1):
        say("pc event schedule", div)
        c, _, d, pop = run(M, ctx, p, schedule=M.PULSE_EVENT, finish_div=div)
        assert np.array_equal(pop, ref.pop) and np.array_equal(c, ref.counts) and d == ref.diag, div


def test_paper_problem_with_population_control(M, ctx, orc):
    """The paper's problem, 1000 batches x 1000 sources, a census at t = 5,
    10, 15 that brings every batch back to 1000 particles on average."""
    p = W.pulse_pc(census_every=5)
    say("paper problem with population control")
    ref = check(orc, p, *run(M, ctx, p), threads=16)
    assert abs(ref.pop[:, :, 1].mean() - 1000) < 5


def test_edge_problems(M, ctx, orc):
    base = W.pulse_pc(n_batches=4, per_batch=60, census_every=4)
    probs = [
        base.with_(pc_target=1),                                       # a batch shrinks to ~1 particle
        base.with_(census_every=1),                                    # a census at every edge
        base.with_(census_every=20),                                   # no census point: the plain problem
        base.with_(scatter=0.0, per_batch=2),                          # batches die out before a census
        base.with_(nu=3.0, scatter=0.3, pc_target=500),                # integer multiplicity, growth by splitting
        base.with_(time_edges=np.array([0.5, 1.0, 2.0, 3.0, 4.5, 6.0]), census_every=2),
        base.with_(x_lo=0.25, x_hi=0.5, sigma_t=2.5, pc_seed=12345),
        base.with_(n_batches=1, per_batch=1, pc_target=7),
    ]
    for i, p in enumerate(probs):
        say("pc edge problem", i)
        check(orc, p, *run(M, ctx, p), threads=4)
    c, f, d, pop = run(M, ctx, probs[2])
    plain = orc.pulse(probs[2], LCG)
    assert pop.shape[1] == 0 and np.array_equal(c, plain.counts) and d == plain.diag


def test_limits(M, ctx, orc):
    """Population control with many copies per arrival (a target far above
    the arrivals), multiplicity near its limit, and 4096 time bins with a
    census every 512."""
    probs = [W.pulse_pc(n_batches=3, per_batch=5, census_every=2, target=5000, t_end=6),
             W.pulse_pc(n_batches=3, per_batch=40, census_every=2, target=60).with_(
                 nu=13.5, scatter=0.5, time_edges=np.array([0.0, 0.25, 0.5, 0.75, 1.0])),
             W.pulse_pc(n_batches=2, per_batch=300, census_every=512, target=250).with_(
                 time_edges=np.linspace(0.0, 20.0, 4097))]
    for i, p in enumerate(probs):
        for sched in (M.PULSE_BANK, M.PULSE_EVENT):
            say("pc limits", i, sched)
            check(orc, p, *run(M, ctx, p, schedule=sched), threads=3)


def test_several_batch_chunks(M, ctx, orc):
    """Runs that go through several chunks of whole batches: many small
    batches (the chunk holds at most 4096), and few large ones."""
    p = W.pulse_pc(n_batches=5000, per_batch=10, census_every=5)
    say("pc chunks: 5000 batches of 10")
    check(orc, p, *run(M, ctx, p), threads=16)
    q = W.pulse_pc(n_batches=5, per_batch=1 << 21, census_every=3, t_end=10)
    say("pc chunks: 5 batches of 2^21")
    c, f, d, pop = run(M, ctx, q)
    for b in (0, 4):
        ref = orc.pulse_pc(q, LCG, b, b + 1)
        assert np.array_equal(c[b], ref.counts[b]), b
        assert np.array_equal(pop[b], ref.pop[b]), b
    particles = d["sources"] + d["secondaries"] + int(pop[:, :, 1].sum())
    assert particles == d["absorbed"] + d["census"] + d["scatters"]
    assert d["draws"] == 2 * (d["sources"] + d["secondaries"]) + int(pop[:, :, 1].sum()) + d["collisions"] + d["scatters"]
