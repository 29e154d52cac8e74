"""Small helpers shared by the GPU tests (tensor <-> NumPy for unsigned
words, which torch supports only partially)."""
import os

import numpy as np


def host_threads(cap=16):
    """Oracle worker threads: the host cores this process may use, at most
    `cap` (the CPU share of one GPU on a shared node)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(cap, n))


def u64_np(t):
    import torch
    return t.contiguous().view(torch.int64).cpu().numpy().view(np.uint64)


def raw_ints(raw):
    """[bins, 2] uint64 tensor of (low, high) words -> list of Python ints."""
    w = u64_np(raw).reshape(-1, 2)
    return [int(lo) | (int(hi) << 64) for lo, hi in w]


def diag_dict(diag, names):
    d = u64_np(diag).reshape(-1, len(names))
    return [dict(zip(names, (int(v) for v in row))) for row in d]


def to_dev_u32(a, dev="cuda:0"):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32)).to(dev)
