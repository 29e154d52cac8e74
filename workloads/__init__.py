"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke
check.

This module holds problem descriptions and NumPy-seeded parameter draws
only: no LCG step, no hash, no skip-ahead and no transport arithmetic, so it
can serve both the CPU oracle and the GPU library without coupling them.

Workloads (each a fixed-source 1-D slab; the source is mono-directional,
mu = +1, at the left face x = 0, t = 0; vacuum on both faces):

* ``small_slab``    20 mfp, sigma_t 1, c 0.9, 20 bins, 1e4 histories, FP64.
* ``draw_counts``   2^26 streams; per-stream draw counts geometric with
                    mean 64 from NumPy seed 42.
* ``long_chain``    50 mfp, sigma_t 1, c 0.99, 200 bins, 1e8 histories,
                    64 batches.
* ``batched``       512 independent slabs from NumPy seed 7: histories
                    log-uniform in [1e3, 1e7], thickness U[5, 50] mfp,
                    sigma_t U[0.5, 2], c U[0.5, 0.99], bins U{20..200}.
* ``multi_region``  10 regions from NumPy seed 11: widths U[1, 5] mfp,
                    sigma_t U[0.2, 3], c U[0.3, 0.995]; 50 space x 20 time
                    bins over [0, 100] (speed 1, census at t = 100);
                    2e8 histories.

Widths "in mfp" are optical thicknesses: the physical width of a region is
its mfp count divided by its sigma_t.

The LCG is X <- (g X + 1) mod 2^63 with g = 2806196910506780709; stride
seeding uses X_0 = 1 and stride Q = 152917, hash seeding the global seed 1.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

G_MCNP = 2806196910506780709
STRIDE_Q = 152917


@dataclass(frozen=True)
class Lcg:
    g: int = G_MCNP
    c: int = 1
    m: int = 63


@dataclass(frozen=True)
class Seeding:
    """How stream i (0-based, offset by first_index) gets its start state.

    kind "stride": X_{Q (first_index + i)} from the base state X_0 = base.
    kind "hash":   hash(first_index + i + 1, parent) with parent = base, or
                   hash(group_key, base) when group_key is given.
    """
    kind: str = "hash"
    base: int = 1
    stride: int = STRIDE_Q
    first_index: int = 0
    group_key: Optional[int] = None


@dataclass
class SlabProblem:
    region_edges: np.ndarray          # float64, n_regions + 1, increasing
    sigma_t: np.ndarray               # float64, n_regions
    scatter: np.ndarray               # float64, n_regions (scattering ratio c)
    bin_edges: np.ndarray             # float64, n_space_bins + 1 (same span)
    n_histories: int
    seeding: Seeding = field(default_factory=Seeding)
    n_batches: int = 1
    time_edges: Optional[np.ndarray] = None   # float64, n_time_bins + 1; last = census

    @property
    def n_space_bins(self) -> int:
        return len(self.bin_edges) - 1

    @property
    def n_time_bins(self) -> int:
        return 0 if self.time_edges is None else len(self.time_edges) - 1

    def with_(self, **kw) -> "SlabProblem":
        return replace(self, **kw)


def homogeneous(width, sigma_t, c, n_bins, n_histories, seeding=None, n_batches=1):
    """One-region slab [0, width] with n_bins equal tally bins."""
    w = float(width)
    be = np.array([w * i / n_bins for i in range(n_bins + 1)], dtype=np.float64)
    be[-1] = w
    return SlabProblem(np.array([0.0, w]), np.array([float(sigma_t)]), np.array([float(c)]), be,
                       int(n_histories), seeding or Seeding(), int(n_batches))


def stride_seeding(first_index=0):
    return Seeding("stride", 1, STRIDE_Q, first_index)


def hash_seeding(first_index=0, group_key=None, base=1):
    return Seeding("hash", base, STRIDE_Q, first_index, group_key)


# ---------------------------------------------------------------- configs

def small_slab(seeding=None, n_histories=10_000):
    return homogeneous(20.0, 1.0, 0.9, 20, n_histories, seeding or hash_seeding())


def draw_counts(n_streams=1 << 26, seed=42, mean=64):
    """Per-stream draw counts, geometric on {1, 2, ...} with the given mean."""
    rng = np.random.default_rng(seed)
    return rng.geometric(1.0 / mean, size=n_streams).astype(np.uint32)


def long_chain(seeding=None, n_histories=100_000_000, n_batches=64):
    return homogeneous(50.0, 1.0, 0.99, 200, n_histories, seeding or hash_seeding(), n_batches)


def batched(n_problems=512, seed=7, seeding_kind="hash", scale=1.0):
    """512 independent slabs.  Hash seeding uses the problem index p + 1 as
    the group key (problem id hashed first); stride seeding gives problem p
    the streams after those of problems 0..p-1.  `scale` shrinks every
    history count (for tests)."""
    rng = np.random.default_rng(seed)
    n_hist = np.floor(10.0 ** rng.uniform(3.0, 7.0, n_problems)).astype(np.int64)
    thick = rng.uniform(5.0, 50.0, n_problems)
    sig = rng.uniform(0.5, 2.0, n_problems)
    c = rng.uniform(0.5, 0.99, n_problems)
    bins = rng.integers(20, 201, n_problems)
    probs = []
    first = 0
    for p in range(n_problems):
        n = max(1, int(n_hist[p] * scale))
        if seeding_kind == "hash":
            sd = hash_seeding(group_key=p + 1)
        else:
            sd = stride_seeding(first)
        first += n
        probs.append(homogeneous(thick[p] / sig[p], sig[p], c[p], int(bins[p]), n, sd))
    return probs


def multi_region(seeding=None, n_histories=200_000_000, seed=11, n_regions=10,
                 n_space_bins=50, n_time_bins=20, census=100.0):
    rng = np.random.default_rng(seed)
    w_mfp = rng.uniform(1.0, 5.0, n_regions)
    sig = rng.uniform(0.2, 3.0, n_regions)
    c = rng.uniform(0.3, 0.995, n_regions)
    re = np.zeros(n_regions + 1)
    re[1:] = np.cumsum(w_mfp / sig)
    L = float(re[-1])
    be = np.array([L * i / n_space_bins for i in range(n_space_bins + 1)], dtype=np.float64)
    be[-1] = L
    te = np.array([census * i / n_time_bins for i in range(n_time_bins + 1)], dtype=np.float64)
    return SlabProblem(re, sig, c, be, int(n_histories), seeding or hash_seeding(), 1, te)


@dataclass
class PulseProblem:
    """Supercritical pulse at x = t = 0 in an infinite homogeneous medium
    (the paper's test problem: scattering ratio 0.4, multiplicity 2.75, run
    to t = 20, collision-estimator flux over x in [-1, 1] in unit time
    bins).  Batch b (0-based) holds `per_batch` sources; its global id is
    first_batch + b.  The seeding's kind, base and stride are used."""
    sigma_t: float = 1.0
    scatter: float = 0.4
    nu: float = 2.75
    x_lo: float = -1.0
    x_hi: float = 1.0
    time_edges: np.ndarray = field(default_factory=lambda: np.arange(21, dtype=np.float64))
    n_batches: int = 1000
    per_batch: int = 1000
    first_batch: int = 0
    seeding: Seeding = field(default_factory=lambda: hash_seeding())
    # population control (hash seeding): a census every `census_every` time
    # bins (0: none), `pc_target` particles per batch after each census,
    # one-off values from the seed `pc_seed`
    census_every: int = 0
    pc_target: int = 0
    pc_seed: int = 2

    @property
    def n_time_bins(self) -> int:
        return len(self.time_edges) - 1

    @property
    def n_sources(self) -> int:
        return self.n_batches * self.per_batch

    def with_(self, **kw) -> "PulseProblem":
        return replace(self, **kw)


def pulse(seeding=None, n_batches=1000, per_batch=1000, first_batch=0):
    """The paper's pulse problem: 1000 batches of 1000 sources by default;
    a study of R repetitions is R x 1000 batches (repetition r holds the
    batches r*1000 .. r*1000+999)."""
    return PulseProblem(n_batches=n_batches, per_batch=per_batch, first_batch=first_batch,
                        seeding=seeding or hash_seeding())


def pulse_few_sources(seeding=None, n_sources=4096, t_end=60):
    """Few sources run long (one batch, unit time bins up to t_end): the
    population grows about e^{0.1 t} (400-fold at t = 60), so a whole
    source family per lane leaves most of the GPU idle while every
    particle of a generation can run in parallel under hash seeding."""
    return PulseProblem(time_edges=np.arange(t_end + 1, dtype=np.float64), n_batches=1,
                        per_batch=n_sources, seeding=seeding or hash_seeding())


def pulse_pc(seeding=None, n_batches=1000, per_batch=1000, census_every=5, target=None, t_end=20):
    """The pulse problem with population control: a census every
    `census_every` unit time bins, after which each batch again holds
    `target` (default: per_batch) particles on average."""
    return PulseProblem(time_edges=np.arange(t_end + 1, dtype=np.float64), n_batches=n_batches,
                        per_batch=per_batch, seeding=seeding or hash_seeding(), census_every=census_every,
                        pc_target=per_batch if target is None else target)


CONFIG_NAMES = {
    "small_slab": "20 mfp slab, c=0.9, 20 bins, 1e4 histories, FP64",
    "draw_counts": "2^26 streams, geometric draw counts (mean 64, seed 42)",
    "long_chain": "50 mfp slab, c=0.99, 200 bins, 1e8 histories, 64 batches",
    "batched": "512 slabs (seed 7), log-uniform 1e3..1e7 histories",
    "multi_region": "10-region slab (seed 11), 50x20 space-time bins, 2e8 histories",
    "pulse": "pulse in an infinite medium, c=0.4, nu=2.75, t<20, 1000 batches x 1000 sources",
}
