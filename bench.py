#!/usr/bin/env python3
"""Benchmark: seeded LCG draws and slab transport on one MI355X.

Step (timed, the headline `value`): one pass of the seed + draw hot path over
the stream microbenchmark workload -- 2^26 streams, per-stream draw counts
geometric with mean 64 (NumPy seed 42), hash seeding with global seed 1,
LCG X <- (g X + 1) mod 2^63.  Every stream is seeded in registers, advanced
count[i] times and its checksum (sum of outputs mod 2^64) written to HBM.
value = RNG draws per second (the draws of the whole step / step time).

Also reported, each timed separately after the headline loop:
  stride        the same workload with stride seeding (X_0 = 1, Q = 152917)
  uniforms      2^26 hash-seeded streams x 16 uniforms written to HBM (GB/s
                against the 8 TB/s peak)
  seed_only     the same 2^26 streams seeded alone: init_streams (states to
                HBM)
  transport     the 1e8-history long-chain slab (50 mfp, c = 0.99, 200 bins,
                64 batches): histories/s, draws/s, events/s for hash FP64,
                hash FP32-flight and stride FP64 (kernel time, HIP events),
                launch options from the library's autotuner (one search per
                precision, reported under "opts")
  pulse         the paper's test problem (pulse in an infinite multiplying
                medium, secondaries seeded on demand), 1000 x 1000 sources:
                hash-seeded generation banks, event-based passes and
                depth-first families against stride-seeded families, and
                the paper's normality study at full size (30 x 1000 batches)
  pulse_population_control
                the same problem with a census every 5 time units that
                brings each batch back to its source count (one-off hashed
                values, copies seeded by eq. 5), against the uncontrolled
                run: time, agreement, figure of merit per time bin
  roofline      of the draw kernel: integer VALU lane-ops per launch over the
                average kernel duration (HIP events on the launch stream)
  batched       512 slabs (seed 7, 5.4e8 histories): one persistent launch
                replayed from a captured hipGraph with autotuned options, FP64
                and FP32-flight, against one run per problem in FP64; the
                FP32 flux error against FP64 per bin, per problem and
                integrated
  multi_region  the 2e8-history 10-region time-dependent slab: history
                schedule FP64 and FP32, event-sorted FP64 (bit-identical)
  transport.roofline, pulse.roofline
                algorithmic VALU lane-operations (counted per event,
                collision and history, or per flight, from the operation
                sequence) over the kernel time (HIP events on the launch
                stream) against the 39.3e12 lane-op/s VALU peak
  cpu_baseline  the CPU oracle on the host cores (at most 16 threads, the
                CPU share of one GPU): the whole draw workload for both
                seedings, every GPU checksum compared with the oracle's;
                single-thread and all-thread rates for draws, the
                long-chain and the multi-region slabs (bounded samples), and
                samples of the pulse problems (the only part of the
                benchmark that uses the oracle)
--only selects legs after the draw legs (for profiling one kernel's workload).

Usage: python bench.py [--gpus 1] [--steps 20] [--warmup 10] [--no-cpu] [--no-transport]
                       [--no-slab] [--no-pulse] [--only LEGS] [--no-autotune] [--copy-probe]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle histories/sec and RNG draws/sec (hash vs stride seeding), % int-VALU peak"

# MI355X: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz = one full-rate 32-bit
# VALU lane-operation per lane per clock.
INT_VALU_PEAK = 256 * 4 * 16 * 2.4e9
# Algorithmic integer lane-ops: a draw is the LCG step on 32-bit halves
# (64-bit low product with the increment, two cross products, one three-way
# add), the reduction to m bits (a mask, or for m = 63 the top bit's
# bookkeeping) and the 64-bit checksum add = 6; a hash seed is
# Listing 1 on a 64-bit key = 16; a stride seed of consecutive streams is
# one k-step affine map from the previous batch base (64-bit multiply-add
# with a 64-bit increment, the mask) = 6.
OPS_PER_DRAW = 6
OPS_PER_HASH_SEED = 16
OPS_PER_STRIDE_SEED = 6
# Slab transport, algorithmic VALU lane-operations, operation by operation:
#   per geometry step (event), FP64, steady: collision distance through the
#     cell's refined reciprocal 3, edge choice by direction 3, numerator 1,
#     edge distance through the flight's reciprocal 3, strict choice 4,
#     quantisation into two 32-bit words 7, tally address 1, optical depth
#     with its clamp 3, move (snap and cell step, or x + mu s and clamps) 4
#   time-dependent: time-edge distance and choice 6, time update 2
#   per collision: LCG step 5, uniform 6, absorption compare 1
#   per scatter: LCG step 5 + uniform 6 for the direction, mu = 2u - 1 2,
#     its refined reciprocal and zero flag 7; the next flight: LCG step 5,
#     uniform 6, logarithm 48 (exponent split 4, reduction 4, a and 2 + a 2,
#     division 8, square 1, degree-10 polynomial 20, the rearranged terms 4,
#     exponent conversion 1, ln 2 terms 4)
#   per history: its stream's start (hash 16 / stride 6), source set-up 6 and
#     its first flight (5 + 6 + 48)
OPS_EVENT = 29
OPS_EVENT_TIMED_EXTRA = 8
OPS_COLLISION = 12
OPS_SCATTER = 5 + 6 + 2 + 7 + 5 + 6 + 48
OPS_HISTORY_HASH = 16 + 6 + 5 + 6 + 48
# Pulse problem, per particle flight: direction (LCG 5, uniform 6, 2u - 1 2),
# flight (LCG 5, uniform 6, logarithm 48, distance through the medium's
# reciprocal 3), census test 2, move x and t 3, collision-estimator window
# and time-bin test 5; per collision: absorption draw and compare 12; per
# scatter: multiplicity draw and count 13; per secondary: its seed (hash of
# the order number and the parent's state) 17
OPS_FLIGHT = 13 + 62 + 2 + 3 + 5
OPS_PULSE_COLLISION = 12
OPS_PULSE_SCATTER = 13
OPS_SECONDARY_HASH = 17


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_threads(cap=16):
    """Oracle worker threads: the host cores this process may use, at most
    `cap` (the CPU share of one GPU on a shared node)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return max(1, min(cap, n))


def draw_workload(M, W, torch, dev, kind, steps, warmup, d_count, n, total_draws, lcg):
    sd = W.hash_seeding() if kind == "hash" else W.stride_seeding()
    chk = torch.empty(n, dtype=torch.uint64, device=dev)
    for _ in range(warmup):
        M.draw(lcg, sd, d_count, chk)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        M.draw(lcg, sd, d_count, chk, stream=stream)
        b.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / steps
    kern_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    return {"ms_per_step": ms_step, "kernel_ms": kern_ms, "draws_per_s": total_draws / (ms_step * 1e-3),
            "chk": chk}


def seed_only_leg(M, W, torch, dev, lcg, n, warmup, reps):
    """Seeding alone over the n streams of the draw workload:
    mcrng_init_streams (every state written to HBM, 8 B each), both
    seedings."""
    st = torch.empty(n, dtype=torch.uint64, device=dev)
    out = {"streams": n}
    for kind in ("hash", "stride"):
        sd = W.hash_seeding() if kind == "hash" else W.stride_seeding()
        for name, fn in (("init_streams", lambda: M.init_streams(lcg, sd, n, st)),):
            for _ in range(warmup):
                fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            out["%s_%s" % (kind, name)] = {"ms": ms, "seeds_per_s": n / (ms * 1e-3),
                                           "hbm_gb_per_s": 8.0 * n / (ms * 1e-3) / 1e9}
    del st
    torch.cuda.empty_cache()
    return out


def uniforms_leg(M, W, torch, dev, lcg, n, k, warmup, reps):
    """mcrng_uniforms over n hash-seeded streams, k numbers each (draw-major
    [k, n] float64): bound by the 8 bytes written per number."""
    u = torch.empty((k, n), dtype=torch.float64, device=dev)
    sd = W.hash_seeding()
    for _ in range(warmup):
        M.uniforms(lcg, sd, u)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        M.uniforms(lcg, sd, u)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = 8.0 * n * k
    # write-only reference on the same buffer: torch's fill kernel
    e0.record()
    for _ in range(reps):
        u.fill_(0.5)
    e1.record()
    torch.cuda.synchronize()
    fill_ms = e0.elapsed_time(e1) / reps
    M.uniforms(lcg, sd, u)
    torch.cuda.synchronize()
    out = {"streams": n, "numbers_per_stream": k, "ms": ms, "numbers_per_s": n * k / (ms * 1e-3),
           "hbm_gb_per_s": nbytes / (ms * 1e-3) / 1e9, "frac_of_hbm_peak": nbytes / (ms * 1e-3) / 8e12,
           "fill_reference_gb_per_s": nbytes / (fill_ms * 1e-3) / 1e9,
           "range_ok": bool(float(u.min()) > 0.0 and float(u.max()) <= 1.0)}
    del u
    torch.cuda.empty_cache()
    return out


def source_sha(*names):
    """sha256 of the named kernel sources (paper_2403_06362_amd/csrc), in order."""
    src = b"".join(open(os.path.join(ROOT, "paper_2403_06362_amd", "csrc", n), "rb").read() for n in names)
    return hashlib.sha256(src).hexdigest()


def traffic_from_profiles(kernel_src_sha, summary="k_draw_hash_2p26_traffic.txt"):
    """HBM bytes per launch measured with rocprofv3 --pmc (FETCH_SIZE, then
    WRITE_SIZE), scaled by a copy kernel of known size; None if absent or
    taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_src_sha:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def transport_leg(M, W, torch, lcg, ctx, prob, opts, reps=2):
    import paper_2403_06362_amd as P
    nb = P.tally_bins([prob])
    raw = torch.empty((nb, 2), dtype=torch.uint64, device="cuda:0")
    flux = torch.empty(nb, dtype=torch.float64, device="cuda:0")
    diag = torch.empty((1, P.NDIAG), dtype=torch.uint64, device="cuda:0")
    ctx.run_histories(lcg, [prob], opts)          # warm-up (and table upload)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        ctx.run_histories(lcg, [prob], opts)
        times.append(ctx.last_run_ms())
    ctx.reduce_tallies(raw, flux, diag)
    torch.cuda.synchronize()
    d = diag.view(torch.int64).cpu().numpy().view(np.uint64)[0]
    dd = dict(zip(P.DIAG_NAMES, (int(v) for v in d)))
    ms = float(np.median(times))
    return {"ms": ms, "kernel": ctx.last_run_kernel(), "histories_per_s": prob.n_histories / (ms * 1e-3),
            "draws_per_s": dd["draws"] / (ms * 1e-3), "events_per_s": dd["events"] / (ms * 1e-3),
            "draws_per_history": dd["draws"] / max(1, dd["histories"]),
            "events_per_history": dd["events"] / max(1, dd["histories"]),
            "flux": flux.cpu().numpy(), "diag": dd}


def transport_ops(diag, timed=False, seeding="hash"):
    """Algorithmic VALU lane-operations of a run, from its diagnostics."""
    scat = diag["collisions"] - diag["absorbed"]
    per_hist = OPS_HISTORY_HASH - (0 if seeding == "hash" else OPS_PER_HASH_SEED - OPS_PER_STRIDE_SEED)
    ev = OPS_EVENT + (OPS_EVENT_TIMED_EXTRA if timed else 0)
    return ev * diag["events"] + OPS_COLLISION * diag["collisions"] + OPS_SCATTER * scat + per_hist * diag["histories"]


def valu_roofline(ops, ms, kernel, unit_counts):
    a = ops / (ms * 1e-3)
    return {"bound": "alu", "achieved": a / 1e12, "peak": INT_VALU_PEAK / 1e12,
            "unit": "Tera VALU lane-ops/s", "frac": a / INT_VALU_PEAK, "traffic": None, "kernel": kernel,
            "algorithmic_ops_per_launch": int(ops), "kernel_ms": ms, "counts": unit_counts}


def flux_errors(f32, f64, sizes):
    """FP32-flight flux against FP64, per problem (sizes = bins of each):
    per-problem L1 (sum |d| / sum f64), integrated (|sum d| / sum f64), and
    per-bin relative error on the bins holding at least 1e-3 of their
    problem's largest bin."""
    l1, integ, binmax, off = [], [], [], 0
    for n in sizes:
        a, b = f32[off:off + n], f64[off:off + n]
        off += n
        tot = b.sum()
        if tot <= 0:
            continue
        d = a - b
        l1.append(float(np.abs(d).sum() / tot))
        integ.append(float(abs(d.sum()) / tot))
        m = b >= 1e-3 * b.max()
        binmax.append(float((np.abs(d[m]) / b[m]).max()))
    l1, integ, binmax = np.array(l1), np.array(integ), np.array(binmax)
    return {"per_problem_l1_max": float(l1.max()), "per_problem_l1_median": float(np.median(l1)),
            "problems_l1_above_1e-6": int(np.sum(l1 > 1e-6)), "problems": int(l1.size),
            "integrated_max": float(integ.max()), "integrated_median": float(np.median(integ)),
            "per_bin_max_on_bins_ge_1e-3_of_max": float(binmax.max())}


def fp32_error(f32, f64, prob):
    """Per-bin error of the FP32-flight flux against the FP64 flux (the
    batch-mean flux over all 1e8 histories), relative and in units of the
    bin's statistical standard error (spread of the 64 batch means)."""
    nb, ns = prob.n_batches, prob.n_space_bins
    a, b = f32.reshape(nb, ns), f64.reshape(nb, ns)
    ma, mb = a.mean(0), b.mean(0)
    se = b.std(0, ddof=1) / np.sqrt(nb)
    m = mb > 0
    rel = np.abs(ma[m] - mb[m]) / mb[m]
    zz = np.abs(ma[m] - mb[m]) / se[m]
    half = ns // 2
    relh = np.abs(ma[:half] - mb[:half]) / mb[:half]
    return {"max_rel": float(rel.max()), "rms_rel": float(np.sqrt(np.mean(rel ** 2))),
            "max_rel_first_half_of_slab": float(relh.max()), "max_in_stat_sigma": float(zz.max()),
            "median_stat_rel_err": float(np.median(se[m] / mb[m]))}


def normality(flux, prob):
    """The paper's normality check, applied to the 64 batch means of every
    bin: Shapiro-Wilk p-values, failures counted at p < 0.05."""
    from scipy import stats
    nb, ns = prob.n_batches, prob.n_space_bins
    a = flux.reshape(nb, ns)
    ps = np.array([stats.shapiro(a[:, i]).pvalue for i in range(ns) if np.ptp(a[:, i]) > 0])
    return {"bins": int(ps.size), "fail_p_lt_0.05": int(np.sum(ps < 0.05)),
            "fail_fraction": float(np.mean(ps < 0.05)), "median_p": float(np.median(ps))}


def rel_err(a, b):
    m = (np.abs(b) > 0)
    r = np.abs(a[m] - b[m]) / np.abs(b[m])
    return float(r.max()) if r.size else 0.0, float(np.sqrt(np.mean(r ** 2))) if r.size else 0.0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-transport", action="store_true", help="headline draw workload only (no slab or pulse legs)")
    ap.add_argument("--no-pulse", action="store_true", help="skip the pulse-problem legs")
    ap.add_argument("--no-slab", action="store_true", help="skip the slab legs (long chain, batched, multi-region)")
    ap.add_argument("--only", default="",
                    help="comma-separated subset of the legs after the draw legs: long_chain, batched, "
                         "multi_region, pulse (schedules), study (the normality study), pulse_pc, "
                         "pulse_bank (the hash-seeded generation banks on 1000 x 1000 alone)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="long-chain legs with the default launch options (no autotuner runs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 512 MiB device copy (reference kernel for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU (--gpus 1); several GPUs are not supported "
              "(the path would shard histories by first_index and all-reduce the integer "
              "tallies).", file=sys.stderr)
        sys.exit(2)

    only = set(x for x in args.only.split(",") if x)
    unknown = only - {"long_chain", "batched", "multi_region", "pulse", "study", "pulse_pc", "pulse_bank"}
    if unknown:
        print("bench.py: unknown legs %s" % ",".join(sorted(unknown)), file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2403_06362_amd as M
    import workloads as W
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    M.lib()
    dev = "cuda:0"
    lcg = W.Lcg()
    n = 1 << 26
    log("generating draw counts")
    counts = W.draw_counts(n, seed=42)
    total_draws = int(counts.sum(dtype=np.uint64))
    d_count = torch.from_numpy(counts).to(dev)

    # the GPU's clocks ramp up over the first tens of milliseconds of sustained
    # work: an untimed spin-up of the same kernels (about half a second) runs
    # before the first leg's warm-up steps, so that the leg measured first is
    # not measured on the ramp
    log("clock spin-up: untimed draws for about 0.5 s")
    spin = torch.empty(n, dtype=torch.uint64, device=dev)
    t_spin = time.perf_counter()
    while time.perf_counter() - t_spin < 0.5:
        for sd in (W.hash_seeding(), W.stride_seeding()):
            M.draw(lcg, sd, d_count, spin)
        torch.cuda.synchronize()
    del spin

    log("headline: hash seeding, %d streams, %d draws" % (n, total_draws))
    hsh = draw_workload(M, W, torch, dev, "hash", args.steps, args.warmup, d_count, n, total_draws, lcg)
    log("stride seeding")
    strd = draw_workload(M, W, torch, dev, "stride", args.steps, args.warmup, d_count, n, total_draws, lcg)

    if args.copy_probe:
        src_t = torch.ones(1 << 27, dtype=torch.float32, device=dev)
        dst_t = torch.empty_like(src_t)
        torch.cuda.synchronize()
        dst_t.copy_(src_t)
        torch.cuda.synchronize()
        del src_t, dst_t

    log("uniforms: 2^26 streams x 16 numbers")
    uni = uniforms_leg(M, W, torch, dev, lcg, n, 16, args.warmup, max(3, args.steps // 4))
    log("seed-only passes")
    seeds = seed_only_leg(M, W, torch, dev, lcg, n, 3, max(3, args.steps // 4))

    chk_hash = hsh["chk"].view(torch.int64).cpu().numpy().view(np.uint64)
    chk_stride = strd["chk"].view(torch.int64).cpu().numpy().view(np.uint64)

    ops_hash = OPS_PER_DRAW * total_draws + OPS_PER_HASH_SEED * n
    ops_stride = OPS_PER_DRAW * total_draws + OPS_PER_STRIDE_SEED * n
    achieved = ops_hash / (hsh["kernel_ms"] * 1e-3)
    traffic = traffic_from_profiles(source_sha("rng_kernels.hip", "device_rng.hpp", "internal.hpp"))
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": INT_VALU_PEAK / 1e12,
                "unit": "Tera int32 VALU lane-ops/s", "frac": achieved / INT_VALU_PEAK,
                "traffic": traffic, "kernel": "k_draw<hash>",
                "algorithmic_ops_per_launch": ops_hash, "kernel_ms": hsh["kernel_ms"],
                "algorithmic_hbm_bytes_per_launch": 12 * n}

    out = {
        "metric": METRIC, "value": hsh["draws_per_s"], "unit": "draws/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": hsh["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "seed+draw microbenchmark: 2^26 streams, geometric draw counts (mean 64, "
                               "seed 42), hash seeding (s=1), LCG g=2806196910506780709 c=1 m=63",
                   "streams": n, "draws_per_step": total_draws, "seeding": "hash"},
        "streams_per_s": n / (hsh["ms_per_step"] * 1e-3),
        "stride_seeding": {"draws_per_s": strd["draws_per_s"], "ms_per_step": strd["ms_per_step"],
                           "kernel_ms": strd["kernel_ms"],
                           "int_valu_frac": ops_stride / (strd["kernel_ms"] * 1e-3) / INT_VALU_PEAK,
                           "hash_over_stride": strd["ms_per_step"] / hsh["ms_per_step"]},
        "uniforms": uni,
        "seed_only": seeds,
        "roofline": roofline,
    }

    def want(leg, slab):
        if args.no_transport or (slab and args.no_slab) or (not slab and args.no_pulse):
            return False
        return not only or leg in only

    if not args.no_transport:
        ctx = M.Context(0)
    if want("long_chain", True):
        prob = W.long_chain()
        # launch options from the library's autotuner, once per precision on
        # the hash-seeded problem (the stride leg reuses the FP64 choice)
        tuned = {}
        for prec in (0, 1):
            if args.no_autotune:
                tuned[prec] = M.make_opts(precision=prec)
                continue
            log("transport long chain: autotune", "fp32" if prec else "fp64")
            tuned[prec], _ = ctx.autotune(lcg, [prob.with_(seeding=W.hash_seeding())], M.make_opts(precision=prec))
        legs = {}
        for name, sd, prec in (("hash_fp64", W.hash_seeding(), 0), ("hash_fp32", W.hash_seeding(), 1),
                               ("stride_fp64", W.stride_seeding(), 0)):
            log("transport long chain", name)
            legs[name] = transport_leg(M, W, torch, lcg, ctx, prob.with_(seeding=sd), tuned[prec])
        tr = {"workload": "long-chain slab: 50 mfp, sigma_t=1, c=0.99, 200 bins, 1e8 histories, 64 batches",
              "opts": {"fp64": tuned[0].as_dict(), "fp32": tuned[1].as_dict()}}
        for k, v in legs.items():
            tr[k] = {kk: vv for kk, vv in v.items() if kk not in ("flux", "diag")}
        tr["fp32_vs_fp64_flux"] = fp32_error(legs["hash_fp32"]["flux"], legs["hash_fp64"]["flux"], prob)
        tr["normality_shapiro_wilk_64_batch_means"] = {
            "hash_fp64": normality(legs["hash_fp64"]["flux"], prob),
            "hash_fp32": normality(legs["hash_fp32"]["flux"], prob),
            "stride_fp64": normality(legs["stride_fp64"]["flux"], prob)}
        tr["fp32_speedup"] = legs["hash_fp64"]["ms"] / legs["hash_fp32"]["ms"]
        tr["hash_over_stride"] = legs["stride_fp64"]["ms"] / legs["hash_fp64"]["ms"]
        d64 = legs["hash_fp64"]["diag"]
        tr["roofline"] = valu_roofline(transport_ops(d64), legs["hash_fp64"]["ms"], "%s<fp64>" % legs["hash_fp64"]["kernel"],
                                       {k: d64[k] for k in ("histories", "events", "collisions", "absorbed")})
        tr["roofline"]["traffic"] = traffic_from_profiles(
            source_sha("transport.hip", "particle.hpp", "device_rng.hpp", "internal.hpp"),
            "k_transport_long_chain_fp64_traffic.txt")
        d32 = legs["hash_fp32"]["diag"]
        tr["roofline_fp32"] = valu_roofline(transport_ops(d32), legs["hash_fp32"]["ms"], "%s<fp32>" % legs["hash_fp32"]["kernel"],
                                            {k: d32[k] for k in ("histories", "events", "collisions", "absorbed")})
        out["histories_per_s"] = legs["hash_fp64"]["histories_per_s"]
        out["transport"] = tr
    if want("batched", True):
        out["batched"] = batched_leg(M, W, torch, lcg, ctx, args.no_autotune)
    if want("multi_region", True):
        out["multi_region"] = multi_region_leg(M, W, torch, lcg, ctx)
    if want("pulse", False) or want("study", False):
        out["pulse"] = pulse_leg(M, W, torch, lcg, ctx, schedules=want("pulse", False), study=want("study", False))
    if want("pulse_pc", False):
        out["pulse_population_control"] = pulse_pc_leg(M, W, torch, lcg, ctx)
    if only and "pulse_bank" in only:
        out["pulse_bank"] = pulse_bank_leg(M, W, torch, lcg, ctx)
    if not args.no_transport:
        ctx.close()

    if not args.no_cpu:
        # the only place the benchmark touches the CPU oracle
        import oracle
        out["cpu_baseline"] = cpu_baseline(oracle, W, lcg, counts, chk_hash, chk_stride, out)

    print(json.dumps(out), flush=True)


def batched_leg(M, W, torch, lcg, ctx, no_autotune=False):
    """512 slabs.  Baseline: the plain FP64 per-problem form, one run (and
    reduce) per problem.  Against it: every problem in one persistent launch
    replayed from a captured hipGraph, launch options from the autotuner,
    in FP64 (bit-identical to the baseline) and FP32-flight (its flux error
    against the FP64 flux per problem and per bin)."""
    import paper_2403_06362_amd as P
    probs = W.batched()
    ntot = sum(p.n_histories for p in probs)
    res = {"workload": "512 slabs (seed 7), log-uniform 1e3..1e7 histories, %d in total" % ntot}
    nb = [P.tally_bins([p]) for p in probs]
    raws = [torch.empty((b, 2), dtype=torch.uint64, device="cuda:0") for b in nb]
    fls = [torch.empty(b, dtype=torch.float64, device="cuda:0") for b in nb]
    log("batched: one run per problem (fp64)")
    ctx1 = M.Context(0)
    ctx1.run_histories(lcg, [probs[0]], M.make_opts())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p, r, f in zip(probs, raws, fls):
        ctx1.run_histories(lcg, [p], M.make_opts())
        ctx1.reduce_tallies(r, f)
    torch.cuda.synchronize()
    per_problem_s = time.perf_counter() - t0
    ctx1.close()
    ref_raw = torch.cat(raws).view(torch.int64).cpu().numpy()
    ref_flux = torch.cat(fls).cpu().numpy()
    res["per_problem_fp64"] = {"s": per_problem_s, "histories_per_s": ntot / per_problem_s}
    tot = P.tally_bins(probs)
    raw = torch.empty((tot, 2), dtype=torch.uint64, device="cuda:0")
    flux = torch.empty(tot, dtype=torch.float64, device="cuda:0")
    diag = torch.empty((len(probs), P.NDIAG), dtype=torch.uint64, device="cuda:0")
    for name, prec in (("fp64", 0), ("fp32", 1)):
        if no_autotune:
            best = M.make_opts(precision=prec)
        else:
            log("batched: autotune", name)
            best, _ = ctx.autotune(lcg, probs, M.make_opts(precision=prec))
        best.use_graph = 1
        ctx.run_histories(lcg, probs, best)
        ctx.reduce_tallies(raw, flux, diag)
        torch.cuda.synchronize()
        times, kms = [], []
        for _ in range(3):
            t0 = time.perf_counter()
            ctx.run_histories(lcg, probs, best)
            ctx.reduce_tallies(raw, flux, diag)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            kms.append(ctx.last_run_ms())
        sec = float(np.median(times))
        leg = {"s": sec, "kernel_ms": float(np.median(kms)), "opts": best.as_dict(), "histories_per_s": ntot / sec,
               "speedup_over_per_problem_fp64": per_problem_s / sec}
        dg = diag.view(torch.int64).cpu().numpy().view(np.uint64).reshape(len(probs), P.NDIAG)
        dd = {k: int(dg[:, i].sum()) for i, k in enumerate(P.DIAG_NAMES) if k != "max_draws"}
        leg["roofline"] = valu_roofline(transport_ops(dd), leg["kernel_ms"], "k_transport<%s> (512 problems)" % name,
                                        {k: dd[k] for k in ("histories", "events", "collisions", "absorbed")})
        if prec == 0:
            leg["bit_identical_to_per_problem"] = bool(np.array_equal(raw.view(torch.int64).cpu().numpy(), ref_raw))
        else:
            leg["flux_error_vs_fp64"] = flux_errors(flux.cpu().numpy(), ref_flux, nb)
        res["persistent_graph_" + name] = leg
    return res


def multi_region_leg(M, W, torch, lcg, ctx):
    prob = W.multi_region()
    res = {"workload": "10-region slab (seed 11), 50x20 space-time bins, 2e8 histories, hash"}
    flux, diag = {}, {}
    for name, opts in (("history_fp64", M.make_opts()), ("history_fp32", M.make_opts(precision=1)),
                       ("event_sorted_fp64", M.make_opts(schedule=1))):
        log("multi region", name)
        r = transport_leg(M, W, torch, lcg, ctx, prob, opts, reps=2)
        res[name] = {k: v for k, v in r.items() if k not in ("flux", "diag")}
        flux[name], diag[name] = r["flux"], r["diag"]
    res["event_sorted_equals_history"] = bool(np.array_equal(flux["event_sorted_fp64"], flux["history_fp64"]))
    res["fp32_error_vs_fp64"] = flux_errors(flux["history_fp32"], flux["history_fp64"], [flux["history_fp64"].size])
    res["fp32_speedup"] = res["history_fp64"]["ms"] / res["history_fp32"]["ms"]
    d = diag["history_fp64"]
    res["roofline"] = valu_roofline(transport_ops(d, timed=True), res["history_fp64"]["ms"],
                                    "%s<fp64, timed>" % res["history_fp64"]["kernel"],
                                    {k: d[k] for k in ("histories", "events", "collisions", "absorbed")})
    return res


def pulse_run(M, torch, lcg, ctx, prob, schedule, reps):
    nt = len(prob.time_edges) - 1
    counts = torch.empty((prob.n_batches, nt), dtype=torch.uint64, device="cuda:0")
    flux = torch.empty((prob.n_batches, nt), dtype=torch.float64, device="cuda:0")
    diag = torch.empty(M.NDIAG, dtype=torch.uint64, device="cuda:0")
    o = M.make_pulse_opts(schedule=schedule)
    times = []
    for _ in range(reps):
        ctx.run_pulse(lcg, prob, counts, flux, diag, o)
        times.append(ctx.last_run_ms())
    d = dict(zip(M.PULSE_DIAG_NAMES, (int(v) for v in diag.view(torch.int64).cpu().numpy())))
    return float(np.median(times)), flux.cpu().numpy(), d


def pulse_pc_run(M, torch, lcg, ctx, prob, reps):
    nt = len(prob.time_edges) - 1
    nc = M.pulse_n_census(prob)
    counts = torch.empty((prob.n_batches, nt), dtype=torch.uint64, device="cuda:0")
    flux = torch.empty((prob.n_batches, nt), dtype=torch.float64, device="cuda:0")
    diag = torch.empty(M.NDIAG, dtype=torch.uint64, device="cuda:0")
    pop = torch.empty((prob.n_batches, nc, 2), dtype=torch.uint64, device="cuda:0")
    times = []
    for _ in range(reps):
        ctx.run_pulse_pc(lcg, prob, counts, flux, diag, pop)
        times.append(ctx.last_run_ms())
    d = dict(zip(M.PULSE_DIAG_NAMES, (int(v) for v in diag.view(torch.int64).cpu().numpy())))
    return float(np.median(times)), flux.cpu().numpy(), d, pop.view(torch.int64).cpu().numpy()


def pulse_pc_leg(M, W, torch, lcg, ctx):
    """Population control with one-off hashed values: the pulse problem with
    a census every 5 time units after which each batch again holds its
    source count on average (copies seeded by eq. 5).  Timed against the
    uncontrolled run; the flux of the two agrees in distribution, and the
    figure of merit 1 / (variance x time) of the batch-mean flux compares
    them per time bin."""
    out = {"workload": "pulse problem (1000 x 1000 sources, census t=20) with population control at t=5,10,15 "
                       "to 1000 particles per batch",
           "few_sources_workload": "4096 sources to t=60 with population control every 5 time units to 4096"}
    p = W.pulse_pc(census_every=5)
    log("pulse population control")
    ms_pc, f_pc, d, pop = pulse_pc_run(M, torch, lcg, ctx, p, 3)
    ms_an, f_an, d_an = pulse_run(M, torch, lcg, ctx, W.pulse(W.hash_seeding()), M.PULSE_BANK, 3)
    copies = int(pop[:, :, 1].sum())
    particles = d["sources"] + d["secondaries"] + copies
    m_pc, m_an = f_pc.mean(0), f_an.mean(0)
    v_pc, v_an = f_pc.var(0, ddof=1) / f_pc.shape[0], f_an.var(0, ddof=1) / f_an.shape[0]
    z = (m_pc - m_an) / np.sqrt(v_pc + v_an)
    fom = (v_an * ms_an) / (v_pc * ms_pc)
    out["paper_problem"] = {
        "ms": ms_pc, "uncontrolled_ms": ms_an, "particles": particles,
        "uncontrolled_particles": d_an["sources"] + d_an["secondaries"],
        "particles_per_s": particles / (ms_pc * 1e-3), "collisions_per_s": d["collisions"] / (ms_pc * 1e-3),
        "arrivals_per_batch_at_census": [float(v) for v in pop[:, :, 0].mean(0)],
        "copies_per_batch_at_census": [float(v) for v in pop[:, :, 1].mean(0)],
        "max_abs_z_vs_uncontrolled": float(np.max(np.abs(z))),
        "fom_ratio_per_time_bin": [float(v) for v in fom]}
    few = W.pulse_few_sources().with_(census_every=5, pc_target=4096)
    log("pulse population control, few sources")
    ms_f, _, d_f, pop_f = pulse_pc_run(M, torch, lcg, ctx, few, 3)
    ms_fa, _, d_fa = pulse_run(M, torch, lcg, ctx, W.pulse_few_sources(), M.PULSE_BANK, 3)
    out["few_sources"] = {
        "ms": ms_f, "uncontrolled_ms": ms_fa,
        "particles": d_f["sources"] + d_f["secondaries"] + int(pop_f[:, :, 1].sum()),
        "uncontrolled_particles": d_fa["sources"] + d_fa["secondaries"],
        "arrivals_at_census": [int(v) for v in pop_f[0, :, 0]]}
    out["sources_per_s"] = p.n_sources / (ms_pc * 1e-3)
    return out


def pulse_leg(M, W, torch, lcg, ctx, schedules=True, study=True):
    """The paper's test problem: a pulse in an infinite medium (c = 0.4,
    nu = 2.75, census t = 20), 1000 batches x 1000 sources; secondaries
    seeded on demand by hashing (eq. 5) or drawing from their source's
    stride stream.  Then the paper's normality study at full size: 30
    repetitions x 1000 batches, Shapiro-Wilk on each of the 20 center-flux
    time points (600 tests per seeding)."""
    out = {"workload": "pulse at x=t=0 in an infinite medium: sigma_t=1, c=0.4, nu=2.75, census t=20, "
                       "collision estimator on x in [-1,1], 20 unit time bins, 1000 batches x 1000 sources",
           "few_sources_workload": "the same medium, one batch of 4096 sources run to t=60 "
                                   "(60 unit time bins, population about 400-fold)"}
    p = W.pulse(W.hash_seeding())
    few = W.pulse_few_sources()
    for tag, base in ((("", p), ("few_sources_", few)) if schedules else ()):
        for name, prob, sched in (("hash_bank", base, M.PULSE_BANK), ("hash_event", base, M.PULSE_EVENT),
                                  ("hash_family", base, M.PULSE_FAMILY),
                                  ("stride_family", base.with_(seeding=W.stride_seeding()), M.PULSE_FAMILY)):
            log("pulse", tag + name)
            ms, _, d = pulse_run(M, torch, lcg, ctx, prob, sched, 3)
            out[tag + name] = {"ms": ms, "sources_per_s": prob.n_sources / (ms * 1e-3),
                               "particles_per_s": (d["sources"] + d["secondaries"]) / (ms * 1e-3),
                               "collisions_per_s": d["collisions"] / (ms * 1e-3),
                               "draws_per_s": d["draws"] / (ms * 1e-3),
                               "collisions_per_source": d["collisions"] / d["sources"], "max_draws": d["max_draws"]}
    if not schedules:
        out["normality_study"] = _study(M, W, torch, lcg, ctx, out) if study else {}
        return out
    out["hash_bank_over_stride_family"] = out["stride_family"]["ms"] / out["hash_bank"]["ms"]
    out["few_sources_hash_bank_over_stride_family"] = (out["few_sources_stride_family"]["ms"] /
                                                       out["few_sources_hash_bank"]["ms"])
    out["hash_family_over_stride_family"] = out["stride_family"]["ms"] / out["hash_family"]["ms"]
    out["hash_event_over_stride_family"] = out["stride_family"]["ms"] / out["hash_event"]["ms"]
    out["few_sources_hash_event_over_stride_family"] = (out["few_sources_stride_family"]["ms"] /
                                                        out["few_sources_hash_event"]["ms"])

    if study:
        out["normality_study"] = _study(M, W, torch, lcg, ctx, out)
    return out


def pulse_ops(d):
    """Algorithmic VALU lane-operations of a pulse run, from its diagnostics."""
    flights = d["sources"] + d["secondaries"]
    return (OPS_FLIGHT * flights + OPS_PULSE_COLLISION * d["collisions"] + OPS_PULSE_SCATTER * d["scatters"]
            + OPS_SECONDARY_HASH * d["secondaries"] + OPS_PER_HASH_SEED * d["sources"]), flights


def pulse_bank_leg(M, W, torch, lcg, ctx, reps=3):
    """The hash-seeded generation banks alone on the paper's 1000 x 1000
    problem (for profiling the bank kernel): run time and the algorithmic
    work per flight over it (the run is a chain of launches with a size
    read-back between generations, so this is a bound on the kernels' rate)."""
    p = W.pulse(W.hash_seeding())
    ms, _, d = pulse_run(M, torch, lcg, ctx, p, M.PULSE_BANK, reps)
    ops, flights = pulse_ops(d)
    out = {"workload": "pulse 1000 x 1000, hash seeding, generation banks", "runs": reps, "ms": ms,
           "sources_per_s": p.n_sources / (ms * 1e-3), "flights": flights}
    out["roofline_over_run_time"] = valu_roofline(ops, ms, "k_pulse_bank + finish (whole run)",
                                                  {"flights": flights, "collisions": d["collisions"],
                                                   "scatters": d["scatters"], "secondaries": d["secondaries"]})
    return out


def _study(M, W, torch, lcg, ctx, out):
    """The paper's normality study at full size: 30 repetitions x 1000
    batches x 1000 sources per seeding, Shapiro-Wilk on each of the 20
    center-flux time points (600 tests per seeding); the hash run's counts
    give the pulse roofline."""
    from scipy import stats
    study = {}
    for kind in ("hash", "stride"):
        sd = W.hash_seeding() if kind == "hash" else W.stride_seeding()
        prob = W.pulse(sd, n_batches=30000)
        log("pulse normality study", kind)
        ms, flux, d = pulse_run(M, torch, lcg, ctx, prob, M.PULSE_AUTO, 1)
        f = flux.reshape(30, 1000, 20)
        pv = np.array([[stats.shapiro(f[r, :, k]).pvalue for k in range(20)] for r in range(30)])
        study[kind] = {"ms": ms, "sources_per_s": prob.n_sources / (ms * 1e-3), "tests": int(pv.size),
                       "fail_p_lt_0.05": int(np.sum(pv < 0.05)),
                       "median_p_per_time_bin": [float(v) for v in np.median(pv, axis=0)],
                       "over_stride_families": d["over_stride"], "max_draws": d["max_draws"]}
        if kind == "hash":
            ops, flights = pulse_ops(d)
            out["roofline"] = valu_roofline(ops, ms, "k_pulse_family (3e7-source study, hash)",
                                            {"flights": flights, "collisions": d["collisions"],
                                             "scatters": d["scatters"], "secondaries": d["secondaries"]})
            out["roofline"]["traffic"] = traffic_from_profiles(
                source_sha("pulse.hip", "pulse.hpp", "device_rng.hpp"), "k_pulse_family_study_traffic.txt")
    study["paper_fails_of_600"] = {"stride": 369, "hash": 339}
    return study


def _rate(fn, units):
    t0 = time.perf_counter()
    fn()
    dt = time.perf_counter() - t0
    return units / dt, dt


def cpu_baseline(oracle, W, lcg, counts, chk_hash, chk_stride, out):
    """The CPU oracle on the host cores: the whole headline draw workload for
    both seedings (timed for hash; every GPU checksum compared with the
    oracle's), single-thread draw, long-chain and multi-region rates on
    bounded samples, all-thread rates beside them, and bounded samples of
    the pulse problems."""
    threads = host_threads()
    ns = counts.size
    draws = int(counts.sum(dtype=np.uint64))
    log("cpu baseline: oracle seed+draw on %d streams, %d threads, 3 passes" % (ns, threads))
    walls, ref = [], None
    for _ in range(3):
        t0 = time.perf_counter()
        r = oracle.seed_and_draw(lcg, W.hash_seeding(), counts, threads=threads)
        walls.append(time.perf_counter() - t0)
        if ref is None:
            ref = r
    dt = float(np.median(walls))
    mism_h = int(np.count_nonzero(ref != chk_hash))
    log("cpu baseline: oracle seed+draw, stride seeding, whole workload")
    ref_s = oracle.seed_and_draw(lcg, W.stride_seeding(), counts, threads=threads)
    mism_s = int(np.count_nonzero(ref_s != chk_stride))
    one = 1 << 21
    r1, _ = _rate(lambda: oracle.seed_and_draw(lcg, W.hash_seeding(), counts[:one], threads=1),
                  int(counts[:one].sum(dtype=np.uint64)))
    res = {"value": draws / dt, "unit": "draws/s", "cores": threads, "kind": "oracle",
           "sample": "the whole workload (%d streams, %d draws), hash seeding, %d threads, 3 passes, median %.2f s "
                     "wall" % (ns, draws, threads, dt),
           "nproc": os.cpu_count(), "threads_used": threads,
           "single_thread_draws_per_s": r1, "single_thread_sample": "first 2^21 streams of the workload",
           "gpu_checksum_mismatches_of_%d" % ns: {"hash": mism_h, "stride": mism_s}}
    if "transport" in out:
        tr = {}
        for name, make, n1, nall in (("long_chain", lambda n: W.long_chain(n_histories=n), 100_000, 1_000_000),
                                     ("multi_region", lambda n: W.multi_region(n_histories=n), 500_000, 4_000_000)):
            log("cpu baseline: oracle", name)
            p1, pa = make(n1), make(nall)
            h1, _ = _rate(lambda: oracle.transport(p1, lcg, threads=1), n1)
            ha, _ = _rate(lambda: oracle.transport(pa, lcg, threads=threads), nall)
            gpu = out["transport"]["hash_fp64"]["histories_per_s"] if name == "long_chain" else \
                out["multi_region"]["history_fp64"]["histories_per_s"]
            tr[name] = {"single_thread_histories_per_s": h1, "single_thread_sample": "first %d histories" % n1,
                        "all_threads_histories_per_s": ha, "threads": threads,
                        "all_threads_sample": "first %d histories" % nall, "gpu_over_all_threads": gpu / ha}
        res["transport"] = tr
    if "pulse" in out and "hash_bank" in out["pulse"]:
        sample = W.pulse(W.hash_seeding(), n_batches=64)
        log("cpu baseline: oracle pulse problem, 64 batches")
        rate, _ = _rate(lambda: oracle.pulse(sample, lcg, threads=threads), sample.n_sources)
        res["pulse"] = {"sources_per_s": rate, "threads": threads, "sample": "64 batches x 1000 sources, hash seeding",
                        "gpu_bank_over_cpu": out["pulse"]["hash_bank"]["sources_per_s"] / rate}
        sample = W.pulse_pc(n_batches=64, census_every=5)
        log("cpu baseline: oracle pulse problem with population control, 64 batches")
        rate, _ = _rate(lambda: oracle.pulse_pc(sample, lcg, threads=threads), sample.n_sources)
        res["pulse_population_control"] = {
            "sources_per_s": rate, "threads": threads, "sample": "64 batches x 1000 sources, census every 5",
            "gpu_over_cpu": out["pulse_population_control"]["sources_per_s"] / rate} \
            if "pulse_population_control" in out else None
    return res


if __name__ == "__main__":
    main()
