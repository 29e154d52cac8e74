"""CPU oracle for the hash- vs stride-seeded LCG transport path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the ``cpu_baseline`` leg of ``bench.py``, never by the library.  The
arithmetic lives in ``mcrng_oracle.c`` (plain C, one history at a time); this
module loads it with ctypes, builds the merged cell geometry with NumPy and
offers a thread-parallel driver over disjoint history ranges whose integer
tallies are summed exactly in Python.

Paper: Cuneo & Variansyah, "An Alternative to Stride-Based RNG for Monte
Carlo Transport" (arXiv 2403.06362).  Which section each routine follows is
stated in the C source.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mcrng_oracle.c")
_LIB = os.path.join(_HERE, "libmcrng_oracle.so")
_lock = threading.Lock()
_lib = None

NDIAG = 10
DIAG_NAMES = ("histories", "leak_left", "leak_right", "absorbed", "census",
              "events", "collisions", "draws", "max_draws", "over_stride")
EV_COLL, EV_EDGE, EV_TIME = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math",
                           "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


class _Lcg(C.Structure):
    _fields_ = [("g", C.c_uint64), ("c", C.c_uint64), ("m", C.c_uint32), ("pad_", C.c_uint32)]


class _Seeding(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("hier", C.c_uint32), ("base", C.c_uint64),
                ("stride", C.c_uint64), ("first_index", C.c_uint64), ("group_key", C.c_uint64)]


class _Problem(C.Structure):
    _fields_ = [("n_cells", C.c_int32), ("n_space_bins", C.c_int32), ("n_time_bins", C.c_int32),
                ("n_batches", C.c_uint32),
                ("edges", C.POINTER(C.c_double)), ("sigma_t", C.POINTER(C.c_double)),
                ("scatter", C.POINTER(C.c_double)), ("bin", C.POINTER(C.c_int32)),
                ("t_edges", C.POINTER(C.c_double)), ("n_histories", C.c_uint64),
                ("lcg", _Lcg), ("seeding", _Seeding)]


class _Event(C.Structure):
    _fields_ = [("type", C.c_int32), ("cell", C.c_int32), ("tbin", C.c_int32),
                ("pad_", C.c_int32), ("s", C.c_double)]


class _Pulse(C.Structure):
    _fields_ = [("sigma_t", C.c_double), ("scatter", C.c_double), ("nu", C.c_double),
                ("x_lo", C.c_double), ("x_hi", C.c_double), ("n_time_bins", C.c_int32),
                ("n_batches", C.c_uint32), ("t_edges", C.POINTER(C.c_double)),
                ("per_batch", C.c_uint64), ("first_batch", C.c_uint64),
                ("lcg", _Lcg), ("seeding", _Seeding),
                ("census_every", C.c_uint32), ("pc_target", C.c_uint64), ("pc_seed", C.c_uint64)]


class _PTrace(C.Structure):
    _fields_ = [("start", C.c_uint64), ("end", C.c_uint64), ("x0", C.c_double), ("t0", C.c_double),
                ("n_out", C.c_uint32), ("draws", C.c_uint32)]


PULSE_DIAG_NAMES = ("sources", "collisions", "tallied", "scatters", "absorbed", "census",
                    "secondaries", "draws", "max_draws", "over_stride")


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
            L = C.CDLL(_LIB)
            u64, u32, dbl = C.c_uint64, C.c_uint32, C.c_double
            P = C.POINTER
            L.orc_lcg_next.argtypes = [u64, u64, u64, u32]; L.orc_lcg_next.restype = u64
            L.orc_skip_coeffs.argtypes = [u64, u64, u64, u32, P(u64), P(u64)]
            L.orc_skip.argtypes = [u64, u64, u64, u64, u32]; L.orc_skip.restype = u64
            L.orc_subhash.argtypes = [u64]; L.orc_subhash.restype = u64
            L.orc_hash.argtypes = [u64, u64]; L.orc_hash.restype = u64
            L.orc_stream_start.argtypes = [P(_Lcg), P(_Seeding), u64]; L.orc_stream_start.restype = u64
            L.orc_init_streams.argtypes = [P(_Lcg), P(_Seeding), u64, C.c_void_p]
            L.orc_seed_and_draw.argtypes = [P(_Lcg), P(_Seeding), u64, C.c_void_p, C.c_void_p, C.c_void_p]
            L.orc_uniform.argtypes = [u64, u32]; L.orc_uniform.restype = dbl
            L.orc_uniforms.argtypes = [P(_Lcg), P(_Seeding), u64, u32, C.c_void_p, C.c_void_p]
            L.orc_ln.argtypes = [dbl]; L.orc_ln.restype = dbl
            L.orc_transport.argtypes = [P(_Problem), C.c_int, u64, u64, C.c_void_p, C.c_void_p, C.c_void_p]
            L.orc_transport.restype = C.c_int
            L.orc_transport_scripted.argtypes = [P(_Problem), C.c_int, C.c_void_p, u64, C.c_void_p,
                                                 C.c_void_p, C.c_void_p, C.c_void_p, u64, P(u64)]
            L.orc_transport_scripted.restype = C.c_int64
            L.orc_u128_to_f64.argtypes = [u64, u64]; L.orc_u128_to_f64.restype = dbl
            L.orc_pulse_run.argtypes = [P(_Pulse), u64, u64, C.c_void_p, C.c_void_p]
            L.orc_pulse_run.restype = C.c_int
            L.orc_pulse_scripted.argtypes = [P(_Pulse), C.c_void_p, u64, C.c_void_p, C.c_void_p]
            L.orc_pulse_scripted.restype = C.c_int64
            L.orc_pulse_flux.argtypes = [P(_Pulse), C.c_void_p, C.c_void_p]
            L.orc_pulse_trace.argtypes = [P(_Pulse), u64, u64, C.c_void_p, C.c_void_p, C.c_void_p, u64, P(u64)]
            L.orc_pulse_trace.restype = C.c_int
            L.orc_pulse_pc_run.argtypes = [P(_Pulse), u64, u64, C.c_void_p, C.c_void_p, C.c_void_p]
            L.orc_pulse_pc_run.restype = C.c_int
            L.orc_pulse_pc_flux.argtypes = [P(_Pulse), C.c_void_p, C.c_void_p, C.c_void_p]
            L.orc_pulse_pc_scripted.argtypes = [P(_Pulse), C.c_void_p, u64, C.c_void_p, C.c_void_p, C.c_void_p,
                                                C.c_void_p, u64, P(u64)]
            L.orc_pulse_pc_scripted.restype = C.c_int64
            L.orc_pulse_pc_census.argtypes = [P(_Pulse), u64, u32, C.c_void_p, C.c_void_p, u64, P(u64), P(u64)]
            L.orc_pulse_pc_census.restype = C.c_int
            _lib = L
    return _lib


# ---------------------------------------------------------------- scalars

def lcg_next(x, g, c, m):
    return int(lib().orc_lcg_next(x, g, c, m))


def skip_coeffs(k, g, c, m):
    G, Cc = C.c_uint64(), C.c_uint64()
    lib().orc_skip_coeffs(k % (1 << 64), g, c, m, C.byref(G), C.byref(Cc))
    return int(G.value), int(Cc.value)


def skip(x0, k, g, c, m):
    return int(lib().orc_skip(x0, k % (1 << 64), g, c, m))


def subhash(x):
    return int(lib().orc_subhash(x))


def hash64(k, s):
    """Listing 1: hash(k, s)."""
    return int(lib().orc_hash(k, s))


def uniform(x, m=63):
    return float(lib().orc_uniform(x, m))


def ln(u):
    return float(lib().orc_ln(u))


def u128_to_f64(v: int) -> float:
    return float(lib().orc_u128_to_f64(v & ((1 << 64) - 1), v >> 64))


# ---------------------------------------------------------------- seeding

def _lcg_struct(lcg):
    return _Lcg(int(lcg.g), int(lcg.c), int(lcg.m), 0)


def _seeding_struct(sd):
    kind = {"stride": 0, "hash": 1}[sd.kind]
    return _Seeding(kind, 1 if sd.group_key is not None else 0, int(sd.base), int(sd.stride),
                    int(sd.first_index), int(sd.group_key or 0))


def stream_start(lcg, seeding, i):
    L, S = _lcg_struct(lcg), _seeding_struct(seeding)
    return int(lib().orc_stream_start(C.byref(L), C.byref(S), i))


def init_streams(lcg, seeding, n):
    out = np.zeros(n, dtype=np.uint64)
    L, S = _lcg_struct(lcg), _seeding_struct(seeding)
    lib().orc_init_streams(C.byref(L), C.byref(S), n, out.ctypes.data)
    return out


def seed_and_draw(lcg, seeding, counts, states=None, threads=1):
    """Checksums (sum of outputs mod 2^64) per stream; seeding=None draws from
    `states` (updated in place with the final states)."""
    counts = np.ascontiguousarray(counts, dtype=np.uint32)
    n = counts.size
    chk = np.zeros(n, dtype=np.uint64)
    L = _lcg_struct(lcg)
    if seeding is None:
        assert states is not None and states.dtype == np.uint64 and states.size == n
        lib().orc_seed_and_draw(C.byref(L), None, n, counts.ctypes.data, states.ctypes.data,
                                chk.ctypes.data)
        return chk

    def part(a, b):
        sd = _seeding_struct(seeding)
        sd.first_index = int(seeding.first_index) + a
        lib().orc_seed_and_draw(C.byref(L), C.byref(sd), b - a, counts[a:].ctypes.data, None,
                                chk[a:].ctypes.data)

    _parallel_ranges(n, threads, part)
    return chk


def uniforms(lcg, seeding, n, k, states=None):
    """[k, n] float64: row j holds every stream's (j+1)-th uniform.  With
    seeding None the start states come from `states` (uint64, updated in
    place to the final states)."""
    L = _lcg_struct(lcg)
    out = np.zeros((k, n), np.float64)
    if seeding is None:
        assert states is not None and states.dtype == np.uint64 and states.size == n
        lib().orc_uniforms(C.byref(L), None, n, k, states.ctypes.data, out.ctypes.data)
    else:
        sd = _seeding_struct(seeding)
        lib().orc_uniforms(C.byref(L), C.byref(sd), n, k, None, out.ctypes.data)
    return out


def _parallel_ranges(n, threads, fn):
    threads = max(1, int(threads))
    if threads == 1 or n < 2 * threads:
        fn(0, n)
        return
    cuts = [n * i // threads for i in range(threads + 1)]
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(lambda i: fn(cuts[i], cuts[i + 1]), range(threads)))


# ---------------------------------------------------------------- geometry

@dataclass
class Cells:
    edges: np.ndarray     # float64, n_cells + 1
    sigma_t: np.ndarray   # float64, n_cells
    scatter: np.ndarray   # float64, n_cells
    bin: np.ndarray       # int32, n_cells


def build_cells(prob) -> Cells:
    """Merge region and tally-bin edges into cells (each cell lies in one
    material region and one space bin)."""
    re = np.asarray(prob.region_edges, dtype=np.float64)
    be = np.asarray(prob.bin_edges, dtype=np.float64)
    if re[0] != be[0] or re[-1] != be[-1]:
        raise ValueError("region and bin edges must span the same interval")
    E = np.union1d(re, be)
    left = E[:-1]
    reg = np.searchsorted(re, left, side="right") - 1
    sb = np.searchsorted(be, left, side="right") - 1
    return Cells(E, np.asarray(prob.sigma_t, np.float64)[reg].copy(),
                 np.asarray(prob.scatter, np.float64)[reg].copy(), sb.astype(np.int32))


def _n_time(prob):
    return 0 if prob.time_edges is None else len(prob.time_edges) - 1


def slice_bins(prob):
    return max(_n_time(prob), 1) * (len(prob.bin_edges) - 1)


def check_track_bound(prob, cells=None):
    """Every track length must stay below 2^7 so that s * 2^56 < 2^63: the
    longest flight is -ln(2^-53) / sigma_t, the longest time step the widest
    time bin."""
    cells = cells or build_cells(prob)
    tau_max = 53 * 0.6931471805599453 + 1e-9
    bound = tau_max / float(np.min(cells.sigma_t))
    if prob.time_edges is not None:
        bound = min(bound, float(np.max(np.diff(np.asarray(prob.time_edges, np.float64)))))
    if not bound < 128.0:
        raise ValueError("track lengths may reach 2^7; the 2^-56 fixed point would overflow")


class _Keep:
    """Holds the NumPy arrays a ctypes problem struct points into."""


def _problem_struct(prob, lcg, cells):
    k = _Keep()
    k.edges = np.ascontiguousarray(cells.edges)
    k.sig = np.ascontiguousarray(cells.sigma_t)
    k.sc = np.ascontiguousarray(cells.scatter)
    k.bin = np.ascontiguousarray(cells.bin, dtype=np.int32)
    nt = _n_time(prob)
    k.te = np.ascontiguousarray(np.asarray(prob.time_edges, np.float64)) if nt else None
    dp = C.POINTER(C.c_double)
    st = _Problem()
    st.n_cells = len(k.sig)
    st.n_space_bins = len(prob.bin_edges) - 1
    st.n_time_bins = nt
    st.n_batches = int(prob.n_batches)
    st.edges = k.edges.ctypes.data_as(dp)
    st.sigma_t = k.sig.ctypes.data_as(dp)
    st.scatter = k.sc.ctypes.data_as(dp)
    st.bin = k.bin.ctypes.data_as(C.POINTER(C.c_int32))
    st.t_edges = k.te.ctypes.data_as(dp) if nt else None
    st.n_histories = int(prob.n_histories)
    st.lcg = _lcg_struct(lcg)
    st.seeding = _seeding_struct(prob.seeding)
    k.st = st
    return k


@dataclass
class Tally:
    """Exact integer track-length sums (units of 2^-56) per
    (batch, time bin, space bin), as Python ints, plus diagnostics."""
    raw: list
    diag: dict
    n_batches: int
    n_time_bins: int
    n_space_bins: int

    def raw_words(self):
        lo = np.array([v & ((1 << 64) - 1) for v in self.raw], dtype=np.uint64)
        hi = np.array([v >> 64 for v in self.raw], dtype=np.uint64)
        return lo, hi


def transport(prob, lcg, float_mode=False, j0=0, j1=None, threads=1) -> Tally:
    """Run histories j0..j1-1 (0-based within the problem) and return their
    exact tallies.  Threads split the range into contiguous pieces; integer
    sums make the result independent of the split."""
    cells = build_cells(prob)
    check_track_bound(prob, cells)
    j1 = int(prob.n_histories) if j1 is None else int(j1)
    nb = int(prob.n_batches)
    nbins = slice_bins(prob) * nb
    keep = _problem_struct(prob, lcg, cells)
    results = []

    def part(a, b):
        lo = np.zeros(nbins, np.uint64)
        hi = np.zeros(nbins, np.uint64)
        dg = np.zeros(NDIAG, np.uint64)
        rc = lib().orc_transport(C.byref(keep.st), 1 if float_mode else 0, j0 + a, j0 + b,
                                 lo.ctypes.data, hi.ctypes.data, dg.ctypes.data)
        if rc != 0:
            raise RuntimeError("oracle transport failed")
        results.append((lo, hi, dg))

    _parallel_ranges(j1 - j0, threads, part)
    raw = [0] * nbins
    diag = np.zeros(NDIAG, dtype=object)
    for lo, hi, dg in results:
        for i in range(nbins):
            raw[i] += (int(hi[i]) << 64) | int(lo[i])
        for i in range(NDIAG):
            diag[i] = max(diag[i], int(dg[i])) if i == 8 else diag[i] + int(dg[i])
    return Tally(raw, dict(zip(DIAG_NAMES, (int(v) for v in diag))), nb, _n_time(prob),
                 len(prob.bin_edges) - 1)


def transport_scripted(prob, lcg, uniforms, float_mode=False, log_cap=4096):
    """One history driven by the given uniforms.  Returns (raw tally list for
    one batch slice, diag dict, events list, uniforms consumed)."""
    cells = build_cells(prob)
    keep = _problem_struct(prob, lcg, cells)
    u = np.ascontiguousarray(uniforms, dtype=np.float64)
    nbins = slice_bins(prob)
    lo = np.zeros(nbins, np.uint64)
    hi = np.zeros(nbins, np.uint64)
    dg = np.zeros(NDIAG, np.uint64)
    log = (_Event * log_cap)()
    nlog = C.c_uint64()
    used = lib().orc_transport_scripted(C.byref(keep.st), 1 if float_mode else 0, u.ctypes.data,
                                        u.size, lo.ctypes.data, hi.ctypes.data, dg.ctypes.data,
                                        log, log_cap, C.byref(nlog))
    events = [(log[i].type, log[i].cell, log[i].tbin, log[i].s)
              for i in range(min(nlog.value, log_cap))]
    raw = [(int(h) << 64) | int(l) for l, h in zip(lo, hi)]
    return raw, dict(zip(DIAG_NAMES, (int(v) for v in dg))), events, int(used)


def batch_sizes(prob):
    """Histories per batch: batch b holds j in [b*bs, (b+1)*bs) with
    bs = ceil(N / n_batches)."""
    n, nb = int(prob.n_histories), int(prob.n_batches)
    bs = max(1, -(-n // nb))
    return [max(0, min(n, (b + 1) * bs) - b * bs) for b in range(nb)]


def flux(prob, tally: Tally, n_per_batch=None):
    """Track-length flux per (batch, time bin, space bin):
    RN(sum q) * 2^-56 / (N_b * dx [* dt]), with N_b the batch's history count
    (or the counts given)."""
    be = np.asarray(prob.bin_edges, np.float64)
    dx = be[1:] - be[:-1]
    nt = _n_time(prob)
    dt = (np.asarray(prob.time_edges, np.float64)[1:] - np.asarray(prob.time_edges, np.float64)[:-1]
          if nt else None)
    nb = int(prob.n_batches)
    n_b = batch_sizes(prob) if n_per_batch is None else list(n_per_batch)
    ntb, nsb = max(nt, 1), len(dx)
    out = np.zeros(nb * ntb * nsb, np.float64)
    for b in range(nb):
        for t in range(ntb):
            for s in range(nsb):
                i = (b * ntb + t) * nsb + s
                r = u128_to_f64(tally.raw[i]) * 2.0 ** -56
                d = float(n_b[b]) * dx[s]
                if nt:
                    d = d * dt[t]
                out[i] = r / d if d != 0.0 else 0.0
    return out


# ---------------------------------------------------------------- pulse problem

def _pulse_struct(prob, lcg):
    k = _Keep()
    k.te = np.ascontiguousarray(prob.time_edges, dtype=np.float64)
    st = _Pulse()
    st.sigma_t, st.scatter, st.nu = float(prob.sigma_t), float(prob.scatter), float(prob.nu)
    st.x_lo, st.x_hi = float(prob.x_lo), float(prob.x_hi)
    st.n_time_bins = len(k.te) - 1
    st.n_batches = int(prob.n_batches)
    st.t_edges = k.te.ctypes.data_as(C.POINTER(C.c_double))
    st.per_batch = int(prob.per_batch)
    st.first_batch = int(prob.first_batch)
    st.lcg = _lcg_struct(lcg)
    st.seeding = _seeding_struct(prob.seeding)
    st.census_every = int(getattr(prob, "census_every", 0))
    st.pc_target = int(getattr(prob, "pc_target", 0))
    st.pc_seed = int(getattr(prob, "pc_seed", 0))
    k.st = st
    return k


@dataclass
class PulseTally:
    counts: np.ndarray   # uint64, (n_batches, n_time_bins)
    diag: dict
    pop: np.ndarray = None   # population control: uint64 (n_batches, n_census, 2): arrivals, copies


def pulse(prob, lcg, b0=0, b1=None, threads=1) -> PulseTally:
    """Collision counts per (batch, time bin) of batches b0 .. b1-1 (the rest
    stay 0) and the diagnostics of those batches."""
    b1 = prob.n_batches if b1 is None else b1
    keep = _pulse_struct(prob, lcg)
    nt = keep.st.n_time_bins

    def part(lo, hi):
        cnt = np.zeros(prob.n_batches * nt, np.uint64)
        dg = np.zeros(NDIAG, np.uint64)
        if lib().orc_pulse_run(C.byref(keep.st), lo, hi, cnt.ctypes.data, dg.ctypes.data) != 0:
            raise ValueError("orc_pulse_run rejected the problem")
        return cnt, dg

    n = b1 - b0
    threads = max(1, min(int(threads), max(n, 1)))
    cuts = [b0 + n * i // threads for i in range(threads + 1)]
    with ThreadPoolExecutor(threads) as ex:
        parts = list(ex.map(lambda i: part(cuts[i], cuts[i + 1]), range(threads)))
    cnt = np.zeros(prob.n_batches * nt, np.uint64)
    dg = np.zeros(NDIAG, np.uint64)
    for c, d in parts:
        cnt += c
        mx = max(dg[8], d[8])
        dg += d
        dg[8] = mx
    return PulseTally(cnt.reshape(prob.n_batches, nt), dict(zip(PULSE_DIAG_NAMES, (int(v) for v in dg))))


def pulse_scripted(prob, lcg, uniforms):
    """One source family driven by the given uniforms (stride semantics).
    Returns (counts per time bin, diag dict, uniforms used)."""
    keep = _pulse_struct(prob, lcg)
    u = np.ascontiguousarray(uniforms, dtype=np.float64)
    cnt = np.zeros(keep.st.n_time_bins, np.uint64)
    dg = np.zeros(NDIAG, np.uint64)
    used = lib().orc_pulse_scripted(C.byref(keep.st), u.ctypes.data, u.size, cnt.ctypes.data, dg.ctypes.data)
    return [int(v) for v in cnt], dict(zip(PULSE_DIAG_NAMES, (int(v) for v in dg))), int(used)


def pulse_flux(prob, lcg, counts):
    keep = _pulse_struct(prob, lcg)
    c = np.ascontiguousarray(counts, dtype=np.uint64).reshape(-1)
    out = np.zeros(c.size, np.float64)
    lib().orc_pulse_flux(C.byref(keep.st), c.ctypes.data, out.ctypes.data)
    return out.reshape(prob.n_batches, keep.st.n_time_bins)


def pulse_trace(prob, lcg, b, i, cap=1 << 16):
    """Source i of batch b alone: (counts per time bin, diag, list of
    per-particle records (start, end, x0, t0, n_out, draws) in processing
    order)."""
    keep = _pulse_struct(prob, lcg)
    cnt = np.zeros(keep.st.n_time_bins, np.uint64)
    dg = np.zeros(NDIAG, np.uint64)
    log = (_PTrace * cap)()
    n = C.c_uint64()
    if lib().orc_pulse_trace(C.byref(keep.st), b, i, cnt.ctypes.data, dg.ctypes.data, log, cap, C.byref(n)) != 0:
        raise ValueError("orc_pulse_trace rejected the problem")
    recs = [(int(log[k].start), int(log[k].end), float(log[k].x0), float(log[k].t0), int(log[k].n_out),
             int(log[k].draws)) for k in range(min(n.value, cap))]
    return [int(v) for v in cnt], dict(zip(PULSE_DIAG_NAMES, (int(v) for v in dg))), recs


# ---------------------------------------------------------------- population control

def pc_n_census(prob):
    """Census points of a population-controlled pulse problem: T[(c+1) K]
    for every (c+1) K < n_time_bins."""
    k = int(prob.census_every)
    return 0 if k == 0 else (prob.n_time_bins - 1) // k


def pulse_pc(prob, lcg, b0=0, b1=None, threads=1) -> PulseTally:
    """The pulse problem with population control at census times (hash
    seeding): counts of batches b0 .. b1-1, diagnostics, and the census
    populations pop[b, c] = (arrivals, copies)."""
    b1 = prob.n_batches if b1 is None else b1
    keep = _pulse_struct(prob, lcg)
    nt = keep.st.n_time_bins
    nc = pc_n_census(prob)

    def part(lo, hi):
        cnt = np.zeros(prob.n_batches * nt, np.uint64)
        dg = np.zeros(NDIAG, np.uint64)
        pop = np.zeros(max(prob.n_batches * nc * 2, 1), np.uint64)
        if lib().orc_pulse_pc_run(C.byref(keep.st), lo, hi, cnt.ctypes.data, dg.ctypes.data, pop.ctypes.data) != 0:
            raise ValueError("orc_pulse_pc_run rejected the problem")
        return cnt, dg, pop

    n = b1 - b0
    threads = max(1, min(int(threads), max(n, 1)))
    cuts = [b0 + n * i // threads for i in range(threads + 1)]
    with ThreadPoolExecutor(threads) as ex:
        parts = list(ex.map(lambda i: part(cuts[i], cuts[i + 1]), range(threads)))
    cnt = np.zeros(prob.n_batches * nt, np.uint64)
    dg = np.zeros(NDIAG, np.uint64)
    pop = np.zeros(max(prob.n_batches * nc * 2, 1), np.uint64)
    for c, d, pp in parts:
        cnt += c
        pop += pp
        mx = max(dg[8], d[8])
        dg += d
        dg[8] = mx
    return PulseTally(cnt.reshape(prob.n_batches, nt), dict(zip(PULSE_DIAG_NAMES, (int(v) for v in dg))),
                      pop[:prob.n_batches * nc * 2].reshape(prob.n_batches, nc, 2))


def pulse_pc_flux(prob, lcg, counts, pop):
    keep = _pulse_struct(prob, lcg)
    c = np.ascontiguousarray(counts, dtype=np.uint64).reshape(-1)
    pp = np.ascontiguousarray(pop, dtype=np.uint64).reshape(-1)
    if pp.size == 0:
        pp = np.zeros(1, np.uint64)
    out = np.zeros(c.size, np.float64)
    lib().orc_pulse_pc_flux(C.byref(keep.st), c.ctypes.data, pp.ctypes.data, out.ctypes.data)
    return out.reshape(prob.n_batches, keep.st.n_time_bins)


def pulse_pc_scripted(prob, lcg, uniforms, cap=1024):
    """One source family driven by the given uniforms (stride semantics) up
    to the first census.  Returns (counts, diag, uniforms used, list of
    census arrivals (x, mu))."""
    keep = _pulse_struct(prob, lcg)
    u = np.ascontiguousarray(uniforms, dtype=np.float64)
    cnt = np.zeros(keep.st.n_time_bins, np.uint64)
    dg = np.zeros(NDIAG, np.uint64)
    cx = np.zeros(cap, np.float64)
    cmu = np.zeros(cap, np.float64)
    n = C.c_uint64()
    used = lib().orc_pulse_pc_scripted(C.byref(keep.st), u.ctypes.data, u.size, cnt.ctypes.data, dg.ctypes.data,
                                       cx.ctypes.data, cmu.ctypes.data, cap, C.byref(n))
    arr = [(float(cx[i]), float(cmu[i])) for i in range(min(n.value, cap))]
    return [int(v) for v in cnt], dict(zip(PULSE_DIAG_NAMES, (int(v) for v in dg))), int(used), arr


def pulse_pc_census(prob, lcg, b, c, cap=1 << 20):
    """Batch b at census c: the arrivals' stream states (in the oracle's
    order) and the start states of the copies leaving it (copy k of
    arrival i after the copies of arrivals 0 .. i-1)."""
    keep = _pulse_struct(prob, lcg)
    arr = np.zeros(cap, np.uint64)
    cop = np.zeros(cap, np.uint64)
    na, nc = C.c_uint64(), C.c_uint64()
    if lib().orc_pulse_pc_census(C.byref(keep.st), b, c, arr.ctypes.data, cop.ctypes.data, cap, C.byref(na),
                                 C.byref(nc)) != 0:
        raise ValueError("orc_pulse_pc_census rejected the problem")
    return [int(v) for v in arr[:min(na.value, cap)]], [int(v) for v in cop[:min(nc.value, cap)]]
