"""GPU parity of the slab transport (mcrng_run_histories +
mcrng_reduce_tallies) against the CPU oracle.

Tallies are exact integers, so the bar is bit-exact raw sums (and bit-exact
flux, whose normalisation is the same operation sequence on both sides),
equal diagnostics, and bit-identical results across launch shapes.  At the
full workload sizes the oracle recomputes every output: all 64 batches of
the 1e8-history long-chain slab (FP64 and FP32), all 512 problems of the
batched set (FP64 and FP32), and the whole 2e8-history multi-region slab
(FP64 and FP32), whose shards and event-sorted run must add up to the same
bits."""
import sys

import numpy as np
import pytest

import workloads as W
from helpers import diag_dict, host_threads, raw_ints

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


def run(M, ctx, probs, **opts):
    import torch
    raw, flux, diag = M.transport(probs, LCG, ctx=ctx, opts=M.make_opts(**opts))
    torch.cuda.synchronize()
    return raw_ints(raw), flux.cpu().numpy(), diag_dict(diag, M.DIAG_NAMES)


def split(values, probs):
    out, off = [], 0
    for p in probs:
        n = p.n_batches * max(p.n_time_bins, 1) * p.n_space_bins
        out.append(values[off:off + n])
        off += n
    return out


def check_parity(orc, probs, raw, flux, diag, float_mode=False, threads=8):
    for p, r, f, d in zip(probs, split(raw, probs), split(list(flux), probs), diag):
        ref = orc.transport(p, LCG, float_mode=float_mode, threads=threads)
        assert r == ref.raw
        assert d == ref.diag
        assert np.array_equal(np.array(f), orc.flux(p, ref))


@pytest.mark.parametrize("kind", ["hash", "stride"])
@pytest.mark.parametrize("precision", [0, 1])
def test_small_slab_parity(M, ctx, orc, kind, precision):
    sd = W.hash_seeding() if kind == "hash" else W.stride_seeding()
    p = W.small_slab(sd)
    say("small slab", kind, precision)
    raw, flux, diag = run(M, ctx, [p], precision=precision)
    check_parity(orc, [p], raw, flux, diag, float_mode=bool(precision))


def test_launch_shapes_bit_identical(M, ctx, orc):
    p = W.homogeneous(10.0, 1.3, 0.95, 37, 20011, W.hash_seeding(), n_batches=3)
    ref = orc.transport(p, LCG, threads=8)
    for block in (64, 256, 1024):
        for hpl in (1, 2, 4):
            for unit in (300, 4096):
                for copies in (1, 2):
                    for cb in (1, 24, 64 * hpl):
                        say("shape", block, hpl, unit, copies, cb)
                        raw, _, diag = run(M, ctx, [p], block=block, hist_per_lane=hpl, unit_histories=unit,
                                           tally_copies=copies, coll_batch=cb)
                        assert raw == ref.raw, (block, hpl, unit, copies, cb)
                        assert diag[0] == ref.diag


@pytest.mark.parametrize("precision", [0, 1])
def test_chained_units_bit_identical(M, ctx, orc, precision, monkeypatch):
    """One problem, one history per lane: the chained kernel (a block holds
    two units and starts the next while the current one's last histories
    finish) gives the oracle's bits and the per-unit kernel's, for units of
    one history up to thousands, fewer units than blocks and many more,
    blocks of one wave up to sixteen, steady and time-dependent slabs, hash
    and stride seeding."""
    cases = [
        (W.homogeneous(10.0, 1.3, 0.95, 37, 20011, W.hash_seeding(), n_batches=3),
         [(256, 0), (64, 1), (256, 7), (1024, 64), (256, 65), (128, 300)]),
        (W.long_chain(W.stride_seeding(), n_histories=30_011, n_batches=5), [(256, 0), (512, 1000)]),
        (W.multi_region(n_histories=20_011, n_space_bins=8, n_time_bins=4), [(256, 0), (256, 97)]),
        (W.small_slab(n_histories=5), [(256, 0), (64, 1)]),
    ]
    for k, (p, shapes) in enumerate(cases):
        ref = orc.transport(p, LCG, float_mode=bool(precision), threads=8)
        for block, unit in shapes:
            say("chained", k, precision, block, unit)
            monkeypatch.setenv("MCRNG_TRANSPORT_CHAIN", "2")
            raw, flux, diag = run(M, ctx, [p], precision=precision, block=block, unit_histories=unit)
            assert ctx.last_run_kernel() == "k_transport_chain"
            assert raw == ref.raw, (k, block, unit)
            assert diag[0] == ref.diag, (k, block, unit)
            assert np.array_equal(flux, orc.flux(p, ref))
            monkeypatch.setenv("MCRNG_TRANSPORT_CHAIN", "0")
            raw0, _, diag0 = run(M, ctx, [p], precision=precision, block=block, unit_histories=unit)
            assert ctx.last_run_kernel() == "k_transport"
            assert raw0 == raw and diag0 == diag
    # graph replays of a chained run (the unit counter and the diagnostic
    # words are cleared by fill kernels inside the graph)
    import torch
    p = cases[0][0]
    monkeypatch.setenv("MCRNG_TRANSPORT_CHAIN", "2")
    eager = run(M, ctx, [p], precision=precision, unit_histories=300)
    for rep in range(3):
        say("chained graph replay", precision, rep)
        g = run(M, ctx, [p], precision=precision, unit_histories=300, use_graph=1)
        assert g[0] == eager[0] and g[2] == eager[2]
        x = torch.ones(1 << 20, device="cuda:0").sum()
        torch.cuda.synchronize()
        assert float(x) == float(1 << 20)
    # two problems, or two histories per lane: not chained
    monkeypatch.setenv("MCRNG_TRANSPORT_CHAIN", "2")
    with pytest.raises(M.McrngError):
        run(M, ctx, [W.small_slab(), W.small_slab()])
    with pytest.raises(M.McrngError):
        run(M, ctx, [W.small_slab()], hist_per_lane=2)


def test_stride_overrun_counted(M, ctx, orc, monkeypatch):
    """Stride seeding with a short stride (Q = 40): many histories draw past
    their Q numbers into the next history's stream (Sec. "Repetition and
    State Space Exhaustion").  Both transport kernels give the oracle's raw
    sums and diagnostics, the count of such histories and the largest draw
    count included."""
    p = W.long_chain(W.Seeding("stride", 7, 40, 3), n_histories=40_009, n_batches=3)
    ref = orc.transport(p, LCG, threads=8)
    assert ref.diag["over_stride"] > 1000 and ref.diag["max_draws"] > 40
    for mode, kernel in (("2", "k_transport_chain"), ("0", "k_transport")):
        monkeypatch.setenv("MCRNG_TRANSPORT_CHAIN", mode)
        say("stride overrun", kernel)
        raw, flux, diag = run(M, ctx, [p], unit_histories=1000)
        assert ctx.last_run_kernel() == kernel
        assert raw == ref.raw and diag[0] == ref.diag
        assert np.array_equal(flux, orc.flux(p, ref))


@pytest.mark.parametrize("precision", [0, 1])
def test_long_chain_parity(M, ctx, orc, precision):
    p = W.long_chain(n_histories=200_003)
    say("long chain 2e5", precision)
    raw, flux, diag = run(M, ctx, [p], precision=precision)
    assert ctx.last_run_kernel() == "k_transport"   # units of 512 histories: too small to chain
    check_parity(orc, [p], raw, flux, diag, float_mode=bool(precision))


@pytest.mark.parametrize("precision", [0, 1])
def test_multi_region_parity(M, ctx, orc, precision):
    p = W.multi_region(n_histories=100_001)
    say("multi region 1e5", precision)
    raw, flux, diag = run(M, ctx, [p], precision=precision)
    check_parity(orc, [p], raw, flux, diag, float_mode=bool(precision))


@pytest.mark.parametrize("kind", ["hash", "stride"])
def test_batched_parity(M, ctx, orc, kind):
    probs = W.batched(seeding_kind=kind, scale=1e-3)
    say("batched 512 (scaled)", kind)
    raw, flux, diag = run(M, ctx, probs)
    check_parity(orc, probs, raw, flux, diag, threads=4)


def test_graph_replays_match_eager(M, ctx, orc):
    import torch
    probs = W.batched(scale=2e-3)[:64]
    eager = run(M, ctx, probs)
    for rep in range(3):
        say("graph replay", rep)
        g = run(M, ctx, probs, use_graph=1)
        assert g[0] == eager[0] and g[2] == eager[2]
        x = torch.ones(1 << 20, device="cuda:0").sum()   # unrelated eager work between replays
        torch.cuda.synchronize()
        assert float(x) == float(1 << 20)
    ref = [orc.transport(p, LCG, threads=4).raw for p in probs[:8]]
    assert split(eager[0], probs)[:8] == ref


@pytest.mark.parametrize("precision", [0, 1])
def test_autotune_choice_legal_cached_and_exact(M, ctx, orc, precision):
    """The autotuner's choice for a reduced batched set and a reduced long
    chain: every option is one the search may pick, a second call returns
    the cached choice without timing, another base option is another cache
    entry, and a run with the chosen options equals the oracle bit for bit
    (and the default options' run)."""
    sets = {"batched": W.batched(scale=2e-3)[:48], "long chain": [W.long_chain(n_histories=300_007)]}
    for name, probs in sets.items():
        say("autotune", name, precision)
        best, ms = ctx.autotune(LCG, probs, M.make_opts(precision=precision))
        d = best.as_dict()
        assert ms > 0.0
        assert d["precision"] == precision and d["schedule"] == 0 and d["use_graph"] == 0
        assert d["block"] in (64, 128, 256, 512, 1024)
        assert d["hist_per_lane"] in (1, 2, 4)
        assert d["tally_copies"] in (1, 2)
        assert d["coll_batch"] in (1, 16, 24, 32, 36, 40, 48)
        assert 256 <= d["unit_histories"] <= (1 << 18)
        assert d["grid"] == 0 and d["bank_size"] == 0 and not any(best.reserved)
        again, ms2 = ctx.autotune(LCG, probs, M.make_opts(precision=precision))
        assert again.as_dict() == d and ms2 == -1.0
        _, ms3 = ctx.autotune(LCG, probs, M.make_opts(precision=precision, grid=256))
        assert ms3 > 0.0   # a different base is a separate search
        tuned = run(M, ctx, probs, **d)
        default = run(M, ctx, probs, precision=precision)
        assert tuned[0] == default[0] and tuned[2] == default[2]
        check_parity(orc, probs, *tuned, float_mode=bool(precision), threads=8)


@pytest.mark.parametrize("precision", [0, 1])
def test_event_schedule_matches_oracle_and_history(M, ctx, orc, precision):
    """Event-sorted schedule (one event per particle per launch, compacted
    bank) gives the history-based schedule's and the oracle's bits."""
    p = W.multi_region(n_histories=60_007)
    ref = orc.transport(p, LCG, float_mode=bool(precision), threads=8)
    hist = run(M, ctx, [p], precision=precision)
    assert hist[0] == ref.raw
    for bank, unit in ((0, 0), (10_000, 3_001), (4_000, 4_096)):
        say("event schedule", precision, bank, unit)
        ev = run(M, ctx, [p], precision=precision, schedule=1, bank_size=bank, unit_histories=unit)
        assert ctx.last_run_kernel() == "k_event_step"
        assert ev[0] == ref.raw, (bank, unit)
        assert ev[2][0] == ref.diag
        assert np.array_equal(ev[1], hist[1])


def test_event_schedule_batched_and_stride(M, ctx, orc):
    probs = W.batched(seeding_kind="stride", scale=5e-4)[:40] + [W.small_slab(n_histories=333)]
    say("event schedule batched")
    ev = run(M, ctx, probs, schedule=1, bank_size=20_000)
    hist = run(M, ctx, probs)
    assert ev[0] == hist[0] and ev[2] == hist[2]
    parts = split(ev[0], probs)
    for i in (0, 7, 40):
        assert parts[i] == orc.transport(probs[i], LCG).raw


def test_event_schedule_tallies_past_the_lds_copy(M, ctx, orc):
    """A block of the event-sorted schedule keeps its home unit's tally in
    LDS only up to 2048 bins; a larger tally is scored straight into HBM.
    A set mixing tallies above, at and below that size gives the oracle's
    bits either way."""
    probs = [W.multi_region(n_histories=20_011, n_space_bins=130, n_time_bins=20),          # 2600 bins
             W.multi_region(n_histories=9_001, seed=5, n_space_bins=128, n_time_bins=16),   # 2048 bins
             W.small_slab(n_histories=5_000)]
    ref = [orc.transport(p, LCG, threads=8).raw for p in probs]
    for bank, unit in ((0, 0), (6_000, 2_000)):
        say("event schedule large tallies", bank, unit)
        ev = run(M, ctx, probs, schedule=1, bank_size=bank, unit_histories=unit)
        assert split(ev[0], probs) == ref, (bank, unit)


def test_event_schedule_slot_low_word_wraps(M, ctx):
    """A slice of one (problem, batch) scores into one slot.  Here 2^24
    histories in one slice each cross about 900 cells of 0.01 mean free
    paths, all in one tally bin: more than 1.2 x 2^33 scores, whose low 32-bit
    halves (uniform below 2^32) add up past 2^64 in the slot's low word.  The
    wrap must reach the high word as a carry: the event-sorted sums equal the
    history schedule's (per-unit slots of 4096 histories, far from wrapping)
    bit for bit."""
    n_cells = 1000
    re = np.arange(n_cells + 1, dtype=np.float64) * 0.01
    p = W.SlabProblem(re, np.ones(n_cells), np.full(n_cells, 0.99), np.array([0.0, re[-1]]), 1 << 24,
                      W.hash_seeding(), 1)
    say("slot wrap: history schedule")
    hist = run(M, ctx, [p])
    assert hist[2][0]["events"] > 1.2 * 2 ** 33
    say("slot wrap: event-sorted, one slice")
    ev = run(M, ctx, [p], schedule=1, bank_size=1 << 24)
    assert ev[0] == hist[0] and ev[2] == hist[2]
    assert np.array_equal(ev[1], hist[1])


def test_zero_histories_and_edge_problems(M, ctx, orc):
    probs = [W.small_slab(n_histories=0), W.small_slab(n_histories=1),
             W.homogeneous(1.0, 2.0, 0.0, 1, 777), W.small_slab(n_histories=64)]
    say("edge problems")
    raw, flux, diag = run(M, ctx, probs)
    check_parity(orc, probs, raw, flux, diag, threads=1)


def test_error_paths(M, ctx):
    p = W.small_slab()
    with pytest.raises(M.McrngError):
        run(M, ctx, [p], block=96)
    with pytest.raises(M.McrngError) as e:   # a unit's tally words bound its size
        run(M, ctx, [p], unit_histories=(1 << 18) + 1)
    assert "unit_histories" in str(e.value)
    run(M, ctx, [p], unit_histories=1 << 18)
    thin = W.homogeneous(100.0, 0.1, 0.5, 10, 10)   # flights up to 367 mfp: fixed point range
    with pytest.raises(M.McrngError) as e:
        run(M, ctx, [thin])
    assert e.value.code == -4


# ------------------------------------------------------------ full sizes

def _batch_raw(raw, p, b):
    n = max(p.n_time_bins, 1) * p.n_space_bins
    return raw[b * n:(b + 1) * n]


@pytest.mark.parametrize("precision", [0, 1])
def test_long_chain_full_size_whole(M, ctx, orc, precision):
    """1e8 histories, 64 batches (the transport benchmark configuration, in
    its default launch options): every batch's raw sums, the flux and the
    diagnostics equal the oracle's whole run."""
    p = W.long_chain()
    say("long chain full", precision)
    raw, flux, diag = run(M, ctx, [p], precision=precision)
    assert ctx.last_run_kernel() == "k_transport_chain"
    say("long chain full: oracle", precision, host_threads())
    ref = orc.transport(p, LCG, float_mode=bool(precision), threads=host_threads())
    bad = [i for i, (a, b) in enumerate(zip(raw, ref.raw)) if a != b]
    assert not bad, (len(bad), bad[:8])
    assert diag[0] == ref.diag
    assert np.array_equal(flux, orc.flux(p, ref))


def test_multi_region_full_size_whole_and_sharded(M, ctx, orc):
    """2e8 histories: the full run equals the oracle's whole run, equals the
    sum of two shards run separately (first_index) with other launch
    shapes, and equals the event-sorted schedule's run."""
    p = W.multi_region()
    say("multi region full")
    raw, flux, diag = run(M, ctx, [p])
    say("multi region full: oracle", host_threads())
    ref = orc.transport(p, LCG, threads=host_threads())
    assert raw == ref.raw and diag[0] == ref.diag
    assert np.array_equal(flux, orc.flux(p, ref))
    h = p.n_histories // 2
    a = p.with_(n_histories=h)
    b = p.with_(n_histories=p.n_histories - h, seeding=W.hash_seeding(first_index=h))
    ra, _, _ = run(M, ctx, [a], block=512, unit_histories=100_000)
    rb, _, _ = run(M, ctx, [b], block=128, hist_per_lane=2)
    assert [x + y for x, y in zip(ra, rb)] == raw
    say("multi region full, event-sorted schedule")
    re_, _, de = run(M, ctx, [p], schedule=1)
    assert re_ == raw and de == diag


def test_multi_region_full_size_fp32_whole(M, ctx, orc):
    """The FP32-flight form of the 2e8-history multi-region slab equals the
    oracle's FP32 mode bit for bit."""
    p = W.multi_region()
    say("multi region full fp32")
    raw, _, diag = run(M, ctx, [p], precision=1)
    say("multi region full fp32: oracle", host_threads())
    ref = orc.transport(p, LCG, float_mode=True, threads=host_threads())
    assert raw == ref.raw and diag[0] == ref.diag


def _oracle_set(orc, probs, float_mode=False):
    """The oracle over a problem set, one problem per worker thread."""
    from concurrent.futures import ThreadPoolExecutor
    order = sorted(range(len(probs)), key=lambda i: -probs[i].n_histories)   # largest first
    with ThreadPoolExecutor(host_threads()) as ex:
        res = dict(zip(order, ex.map(lambda i: orc.transport(probs[i], LCG, float_mode=float_mode), order)))
    return [res[i] for i in range(len(probs))]


@pytest.mark.parametrize("precision", [0, 1])
def test_batched_full_size_whole(M, ctx, orc, precision):
    """512 problems, 5.4e8 histories in one persistent launch: every
    problem's raw sums and diagnostics equal the oracle's (including the
    1e6-1e7-history problems that load the persistent scheduler)."""
    probs = W.batched()
    say("batched full", precision)
    raw, flux, diag = run(M, ctx, probs, precision=precision)
    say("batched full: oracle", precision, host_threads())
    refs = _oracle_set(orc, probs, float_mode=bool(precision))
    parts = split(raw, probs)
    fparts = split(list(flux), probs)
    for i, ref in enumerate(refs):
        assert parts[i] == ref.raw, i
        assert diag[i] == ref.diag, i
        assert np.array_equal(np.array(fparts[i]), orc.flux(probs[i], ref)), i
