"""ctypes binding of libmcrng.so (include/mcrng.h): argument marshalling only.

Device buffers are torch tensors on a ROCm device (`.data_ptr()` is passed
through); streams are torch streams (their `.cuda_stream` handle).  Every
computation happens in the library's HIP kernels.  The library must have
been built (paper_2403_06362_amd/build.py); without it every entry point
raises.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmcrng.so")

OK = 0
WSTRIDE_WRAP = 1
EINVAL, ENOMEM, EDEVICE, ERANGE, ESTATE = -1, -2, -3, -4, -5
SEED_STRIDE, SEED_HASH = 0, 1
FP64, FP32 = 0, 1
SCHED_HISTORY, SCHED_EVENT = 0, 1
PULSE_AUTO, PULSE_BANK, PULSE_FAMILY, PULSE_EVENT = 0, 1, 2, 3
NDIAG = 10
DIAG_NAMES = ("histories", "leak_left", "leak_right", "absorbed", "census",
              "events", "collisions", "draws", "max_draws", "over_stride")
PULSE_DIAG_NAMES = ("sources", "collisions", "tallied", "scatters", "absorbed", "census",
                    "secondaries", "draws", "max_draws", "over_stride")

# every symbol include/mcrng.h declares
EXPORTS = ("mcrng_init_streams", "mcrng_draw", "mcrng_ctx_create", "mcrng_ctx_destroy",
           "mcrng_tally_bins", "mcrng_run_histories", "mcrng_reduce_tallies", "mcrng_autotune",
           "mcrng_last_run_ms", "mcrng_last_error", "mcrng_version", "mcrng_run_pulse", "mcrng_uniforms",
           "mcrng_run_pulse_pc", "mcrng_run_histories_noalloc", "mcrng_last_run_kernel")


class McrngError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("mcrng error %d: %s" % (code, msg))
        self.code = code


class Lcg(C.Structure):
    _fields_ = [("g", C.c_uint64), ("c", C.c_uint64), ("m", C.c_uint32), ("reserved", C.c_uint32)]


class Seeding(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("hier", C.c_uint32), ("base", C.c_uint64),
                ("stride", C.c_uint64), ("first_index", C.c_uint64), ("group_key", C.c_uint64)]


class Problem(C.Structure):
    _fields_ = [("n_regions", C.c_uint32), ("n_space_bins", C.c_uint32), ("n_time_bins", C.c_uint32),
                ("n_batches", C.c_uint32), ("region_edges", C.POINTER(C.c_double)),
                ("sigma_t", C.POINTER(C.c_double)), ("scatter", C.POINTER(C.c_double)),
                ("bin_edges", C.POINTER(C.c_double)), ("time_edges", C.POINTER(C.c_double)),
                ("n_histories", C.c_uint64), ("seeding", Seeding)]


class RunOpts(C.Structure):
    _fields_ = [("precision", C.c_uint32), ("schedule", C.c_uint32), ("block", C.c_uint32),
                ("hist_per_lane", C.c_uint32), ("unit_histories", C.c_uint32), ("grid", C.c_uint32),
                ("tally_copies", C.c_uint32), ("use_graph", C.c_uint32), ("bank_size", C.c_uint32),
                ("coll_batch", C.c_uint32), ("reserved", C.c_uint32 * 6)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_ if k != "reserved"}


class PulseProblem(C.Structure):
    _fields_ = [("sigma_t", C.c_double), ("scatter", C.c_double), ("multiplicity", C.c_double),
                ("x_lo", C.c_double), ("x_hi", C.c_double), ("n_time_bins", C.c_uint32),
                ("n_batches", C.c_uint32), ("time_edges", C.POINTER(C.c_double)),
                ("per_batch", C.c_uint64), ("first_batch", C.c_uint64), ("seeding", Seeding)]


class PulsePc(C.Structure):
    _fields_ = [("census_every", C.c_uint32), ("reserved0", C.c_uint32), ("target", C.c_uint64),
                ("seed", C.c_uint64), ("reserved", C.c_uint64 * 2)]


class PulseOpts(C.Structure):
    _fields_ = [("schedule", C.c_uint32), ("block", C.c_uint32), ("stack_depth", C.c_uint32),
                ("finish_div", C.c_uint32), ("chunk", C.c_uint32), ("reserved", C.c_uint32 * 3)]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libmcrng.so is not built: run `python -m paper_2403_06362_amd.build` "
                              "(or __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        vp, u64, u32, i32 = C.c_void_p, C.c_uint64, C.c_uint32, C.c_int
        P = C.POINTER
        L.mcrng_init_streams.argtypes = [P(Lcg), P(Seeding), u64, vp, vp]
        L.mcrng_draw.argtypes = [P(Lcg), P(Seeding), u64, vp, vp, vp, vp]
        L.mcrng_ctx_create.argtypes = [i32, P(vp)]
        L.mcrng_ctx_destroy.argtypes = [vp]
        L.mcrng_tally_bins.argtypes = [P(Problem), u32]
        L.mcrng_tally_bins.restype = u64
        L.mcrng_run_histories.argtypes = [vp, P(Lcg), P(Problem), u32, P(RunOpts), vp]
        L.mcrng_reduce_tallies.argtypes = [vp, vp, vp, vp, vp]
        L.mcrng_autotune.argtypes = [vp, P(Lcg), P(Problem), u32, P(RunOpts), P(RunOpts), P(C.c_float), vp]
        L.mcrng_last_run_ms.argtypes = [vp]
        L.mcrng_last_run_ms.restype = C.c_float
        L.mcrng_last_run_kernel.argtypes = [vp]
        L.mcrng_last_run_kernel.restype = C.c_char_p
        L.mcrng_last_error.argtypes = []
        L.mcrng_last_error.restype = C.c_char_p
        L.mcrng_version.argtypes = []
        L.mcrng_run_pulse.argtypes = [vp, P(Lcg), P(PulseProblem), P(PulseOpts), vp, vp, vp, vp]
        L.mcrng_uniforms.argtypes = [P(Lcg), P(Seeding), u64, u32, vp, vp, vp]
        L.mcrng_run_pulse_pc.argtypes = [vp, P(Lcg), P(PulseProblem), P(PulsePc), P(PulseOpts), vp, vp, vp, vp, vp]
        L.mcrng_run_histories_noalloc.argtypes = [P(Lcg), P(Problem), u32, P(RunOpts), vp, vp, vp, vp]
        for name in EXPORTS:
            if name not in ("mcrng_tally_bins", "mcrng_last_run_ms", "mcrng_last_error", "mcrng_last_run_kernel"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc < 0:
        raise McrngError(rc, lib().mcrng_last_error().decode())
    return rc


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def _ptr(t, dtype=None, n=None, what="tensor"):
    """Device pointer of a contiguous torch tensor (checked, not converted)."""
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("%s must be a contiguous device tensor" % what)
    if dtype is not None and t.dtype != dtype:
        raise ValueError("%s must have dtype %s" % (what, dtype))
    if n is not None and t.numel() < n:
        raise ValueError("%s holds %d elements, needs %d" % (what, t.numel(), n))
    return C.c_void_p(t.data_ptr())


def make_lcg(lcg):
    return Lcg(int(lcg.g), int(lcg.c), int(lcg.m), 0)


def make_seeding(sd):
    kind = {"stride": SEED_STRIDE, "hash": SEED_HASH}[sd.kind] if isinstance(sd.kind, str) else int(sd.kind)
    gk = getattr(sd, "group_key", None)
    return Seeding(kind, 0 if gk is None else 1, int(sd.base), int(sd.stride), int(sd.first_index),
                   0 if gk is None else int(gk))


def make_opts(**kw):
    o = RunOpts()
    for k, v in kw.items():
        if v is not None:
            setattr(o, k, int(v))
    return o


class _Arrays:
    """Keeps the host arrays a problem struct points into alive."""


def make_problems(problems):
    import numpy as np
    keep = []
    arr = (Problem * len(problems))()
    dp = C.POINTER(C.c_double)
    for i, pr in enumerate(problems):
        k = _Arrays()
        k.re = np.ascontiguousarray(pr.region_edges, dtype=np.float64)
        k.sig = np.ascontiguousarray(pr.sigma_t, dtype=np.float64)
        k.sc = np.ascontiguousarray(pr.scatter, dtype=np.float64)
        k.be = np.ascontiguousarray(pr.bin_edges, dtype=np.float64)
        k.te = None if pr.time_edges is None else np.ascontiguousarray(pr.time_edges, dtype=np.float64)
        keep.append(k)
        s = arr[i]
        s.n_regions = len(k.sig)
        s.n_space_bins = len(k.be) - 1
        s.n_time_bins = 0 if k.te is None else len(k.te) - 1
        s.n_batches = int(pr.n_batches)
        s.region_edges = k.re.ctypes.data_as(dp)
        s.sigma_t = k.sig.ctypes.data_as(dp)
        s.scatter = k.sc.ctypes.data_as(dp)
        s.bin_edges = k.be.ctypes.data_as(dp)
        s.time_edges = None if k.te is None else k.te.ctypes.data_as(dp)
        s.n_histories = int(pr.n_histories)
        s.seeding = make_seeding(pr.seeding)
    return arr, keep


# ------------------------------------------------------------ entry points

def init_streams(lcg, seeding, n, d_state, stream=None):
    """mcrng_init_streams: start states of n streams into d_state (uint64 tensor)."""
    import torch
    L, S = make_lcg(lcg), make_seeding(seeding)
    return _check(lib().mcrng_init_streams(C.byref(L), C.byref(S), int(n),
                                           _ptr(d_state, torch.uint64, n, "d_state"), _stream(stream)))


def draw(lcg, seeding, d_count, d_checksum, d_state=None, stream=None):
    """mcrng_draw: advance n = d_count.numel() streams; checksums into d_checksum."""
    import torch
    n = d_count.numel()
    L = make_lcg(lcg)
    S = None if seeding is None else C.byref(make_seeding(seeding))
    return _check(lib().mcrng_draw(C.byref(L), S, n, _ptr(d_count, torch.uint32, n, "d_count"),
                                   _ptr(d_state, torch.uint64, n, "d_state"),
                                   _ptr(d_checksum, torch.uint64, n, "d_checksum"), _stream(stream)))


def make_pulse_problem(pr):
    """ctypes struct of a workloads.PulseProblem-like object (and the host
    array it points into, to keep alive)."""
    import numpy as np
    te = np.ascontiguousarray(pr.time_edges, dtype=np.float64)
    sd = make_seeding(pr.seeding)
    sd.hier, sd.first_index, sd.group_key = 0, 0, 0
    st = PulseProblem(float(pr.sigma_t), float(pr.scatter), float(pr.nu), float(pr.x_lo), float(pr.x_hi),
                      len(te) - 1, int(pr.n_batches), te.ctypes.data_as(C.POINTER(C.c_double)),
                      int(pr.per_batch), int(pr.first_batch), sd)
    return st, te


def make_pulse_pc(pr):
    """mcrng_pulse_pc of a workloads.PulseProblem-like object (census_every,
    pc_target, pc_seed)."""
    return PulsePc(int(pr.census_every), 0, int(pr.pc_target), int(pr.pc_seed))


def pulse_n_census(pr):
    k = int(pr.census_every)
    return 0 if k == 0 else (len(pr.time_edges) - 2) // k


def make_pulse_opts(**kw):
    o = PulseOpts()
    for k, v in kw.items():
        if v is not None:
            setattr(o, k, int(v))
    return o


def uniforms(lcg, seeding, d_u, d_state=None, stream=None):
    """mcrng_uniforms: d_u is a float64 tensor [k, n] (row j holds every
    stream's (j+1)-th number)."""
    import torch
    if d_u.dim() != 2:
        raise ValueError("d_u must be a [k, n] tensor")
    k, n = int(d_u.shape[0]), int(d_u.shape[1])
    L = make_lcg(lcg)
    S = None if seeding is None else C.byref(make_seeding(seeding))
    return _check(lib().mcrng_uniforms(C.byref(L), S, n, k, _ptr(d_state, torch.uint64, n, "d_state"),
                                       _ptr(d_u, torch.float64, n * k, "d_u"), _stream(stream)))


def run_histories_noalloc(lcg, problems, d_raw, d_flux, d_diag=None, opts=None, stream=None):
    """mcrng_run_histories_noalloc: run and reduce in one call, no device
    allocation by the library (its static scratch holds the run)."""
    import torch
    arr, _keep = make_problems(problems)
    nb = int(lib().mcrng_tally_bins(arr, len(problems)))
    L = make_lcg(lcg)
    o = opts if opts is not None else RunOpts()
    return _check(lib().mcrng_run_histories_noalloc(C.byref(L), arr, len(problems), C.byref(o),
                                                    _ptr(d_raw, torch.uint64, 2 * nb, "d_raw"),
                                                    _ptr(d_flux, torch.float64, nb, "d_flux"),
                                                    _ptr(d_diag, torch.uint64, len(problems) * NDIAG, "d_diag"),
                                                    _stream(stream)))


def tally_bins(problems):
    arr, _keep = make_problems(problems)
    return int(lib().mcrng_tally_bins(arr, len(problems)))


class Context:
    """An mcrng_ctx bound to one device."""

    def __init__(self, device=0):
        self._h = C.c_void_p()
        _check(lib().mcrng_ctx_create(int(device), C.byref(self._h)))

    def close(self):
        if self._h:
            lib().mcrng_ctx_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run_histories(self, lcg, problems, opts=None, stream=None):
        arr, _keep = make_problems(problems)
        L = make_lcg(lcg)
        o = opts if opts is not None else RunOpts()
        return _check(lib().mcrng_run_histories(self._h, C.byref(L), arr, len(problems), C.byref(o),
                                                _stream(stream)))

    def reduce_tallies(self, d_raw, d_flux, d_diag=None, stream=None):
        import torch
        return _check(lib().mcrng_reduce_tallies(self._h, _ptr(d_raw, torch.uint64, None, "d_raw"),
                                                 _ptr(d_flux, torch.float64, None, "d_flux"),
                                                 _ptr(d_diag, torch.uint64, None, "d_diag"), _stream(stream)))

    def autotune(self, lcg, problems, base=None, stream=None):
        arr, _keep = make_problems(problems)
        L = make_lcg(lcg)
        b = base if base is not None else RunOpts()
        best = RunOpts()
        ms = C.c_float()
        _check(lib().mcrng_autotune(self._h, C.byref(L), arr, len(problems), C.byref(b), C.byref(best),
                                    C.byref(ms), _stream(stream)))
        return best, float(ms.value)

    def run_pulse(self, lcg, problem, d_counts, d_flux=None, d_diag=None, opts=None, stream=None):
        """mcrng_run_pulse (returns after the run has finished)."""
        import torch
        st, _te = make_pulse_problem(problem)
        L = make_lcg(lcg)
        o = opts if opts is not None else PulseOpts()
        n = int(problem.n_batches) * (len(_te) - 1)
        return _check(lib().mcrng_run_pulse(self._h, C.byref(L), C.byref(st), C.byref(o),
                                            _ptr(d_counts, torch.uint64, n, "d_counts"),
                                            _ptr(d_flux, torch.float64, n, "d_flux"),
                                            _ptr(d_diag, torch.uint64, NDIAG, "d_diag"), _stream(stream)))

    def run_pulse_pc(self, lcg, problem, d_counts, d_flux=None, d_diag=None, d_pop=None, opts=None, stream=None):
        """mcrng_run_pulse_pc: the pulse problem with population control
        (problem.census_every, pc_target, pc_seed); d_pop is a uint64 tensor
        [n_batches, n_census, 2] or None.  Returns after the run."""
        import torch
        st, _te = make_pulse_problem(problem)
        L = make_lcg(lcg)
        pc = make_pulse_pc(problem)
        o = opts if opts is not None else PulseOpts()
        n = int(problem.n_batches) * (len(_te) - 1)
        npop = int(problem.n_batches) * pulse_n_census(problem) * 2
        return _check(lib().mcrng_run_pulse_pc(self._h, C.byref(L), C.byref(st), C.byref(pc), C.byref(o),
                                               _ptr(d_counts, torch.uint64, n, "d_counts"),
                                               _ptr(d_flux, torch.float64, n, "d_flux"),
                                               _ptr(d_diag, torch.uint64, NDIAG, "d_diag"),
                                               _ptr(d_pop, torch.uint64, npop, "d_pop"), _stream(stream)))

    def last_run_ms(self):
        return float(lib().mcrng_last_run_ms(self._h))

    def last_run_kernel(self):
        return lib().mcrng_last_run_kernel(self._h).decode()
