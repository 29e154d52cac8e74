"""Pins of the oracle's transport half.

* Scripted trajectories: one history driven by chosen uniforms, events and
  tallies derived by hand (edge crossings, snapping, collisions, leaks on
  both faces, mu = 0, time steps and census, cross-section changes between
  regions).
* Closed forms: a pure absorber's track length per bin is
  (exp(-S a) - exp(-S b)) / S and its transmission exp(-S L); in a time-
  dependent pure absorber at speed 1 a particle is at x = t, which fixes the
  space-time tally and the census fraction.
* Half-space albedo for isotropic scattering and normal incidence:
  1 - sqrt(1 - c) H(1), with Chandrasekhar's H-function solved here from
  its integral equation; also for a slab split into identical regions.
* Exact particle balance; collision-estimator identity
  E[sum sigma_t * track] = E[collisions] (both estimate the collision rate).
* Integer tallies are independent of threads, sharding and batching.
* Flux normalisation: a transparent time-dependent slab (every history's
  track per space-time bin is the bin's x = t overlap, so the flux is that
  overlap / (dx dt) exactly, for every batch whatever its size), and a
  time-dependent pure absorber whose per-batch flux meets the closed-form
  mean track / (dx dt) within 5 standard errors.
"""
import math

import numpy as np
import pytest

import workloads as W

LCG = W.Lcg()
Q56 = 2.0 ** 56


def qexact(s):
    v = s * Q56
    r = math.floor(v)
    frac = v - r
    if frac > 0.5 or (frac == 0.5 and r % 2 == 1):
        r += 1
    return int(r)


def slab(edges, sig, c, bins, n=1, time_edges=None, n_batches=1, seeding=None):
    return W.SlabProblem(np.array(edges, float), np.array(sig, float), np.array(c, float),
                         np.array(bins, float), n, seeding or W.hash_seeding(), n_batches,
                         None if time_edges is None else np.array(time_edges, float))


# ------------------------------------------------------------ scripted histories

def test_scripted_edges_then_scatter_then_absorb(orc):
    p = slab([0, 4], [1.0], [0.5], [0, 1, 2, 3, 4])
    tau0 = -orc.ln(0.125)
    raw, d, ev, used = orc.transport_scripted(p, LCG, [0.125, 0.25, 0.125, 0.5, 0.75])
    assert used == 5 and d["absorbed"] == 1 and d["draws"] == 5 and d["collisions"] == 2
    kinds = [e[0] for e in ev]
    assert kinds == [1, 1, 0, 1, 0]                    # edge, edge, collision, edge, collision
    assert [e[1] for e in ev] == [0, 1, 2, 2, 1]
    s3 = (tau0 - 1.0) - 1.0                            # remaining depth after two unit cells
    x3 = 2.0 + 1.0 * s3
    mu = 2.0 * 0.125 - 1.0                             # -0.75
    tau = -orc.ln(0.5)
    s4 = (2.0 - x3) / mu                               # back to the edge at x = 2
    s5 = tau - 1.0 * s4
    assert [e[3] for e in ev] == [1.0, 1.0, s3, s4, s5]
    assert raw == [qexact(1.0), qexact(1.0) + qexact(s5), qexact(s3) + qexact(s4), 0]


def test_scripted_leak_right_and_left(orc):
    p = slab([0, 2], [1.0], [0.9], [0, 1, 2])
    raw, d, ev, used = orc.transport_scripted(p, LCG, [2.0 ** -53])
    assert d["leak_right"] == 1 and used == 1 and [e[0] for e in ev] == [1, 1]
    assert raw == [qexact(1.0), qexact(1.0)]
    p = slab([0, 3], [1.0], [0.9], [0, 1, 2, 3])
    raw, d, ev, used = orc.transport_scripted(p, LCG, [0.5, 0.1, 2.0 ** -53, 2.0 ** -53])
    assert d["leak_left"] == 1 and used == 4
    x = 0.0 + 1.0 * (-orc.ln(0.5))
    mu = 2.0 * 2.0 ** -53 - 1.0
    se = (0.0 - x) / mu
    assert [e[0] for e in ev] == [0, 1]
    assert raw == [qexact(-orc.ln(0.5)) + qexact(se), 0, 0]


def test_scripted_zero_direction(orc):
    # mu = 2 * 0.5 - 1 = 0: no edge distance, the particle collides in place
    p = slab([0, 2], [2.0], [0.9], [0, 1, 2])
    u = [0.5, 0.1, 0.5, 0.25, 0.95]
    raw, d, ev, used = orc.transport_scripted(p, LCG, u)
    assert used == 5 and d["absorbed"] == 1
    assert [e[0] for e in ev] == [0, 0]
    s1 = (-orc.ln(0.5)) / 2.0
    s2 = (-orc.ln(0.25)) / 2.0
    assert [e[3] for e in ev] == [s1, s2]
    assert raw == [qexact(s1) + qexact(s2), 0]


def test_scripted_time_steps_and_census(orc):
    p = slab([0, 10], [1.0], [1.0], [0, 5, 10], time_edges=[0, 1, 2, 3])
    raw, d, ev, used = orc.transport_scripted(p, LCG, [2.0 ** -53])
    assert d["census"] == 1 and used == 1
    assert [e[0] for e in ev] == [2, 2, 2]
    # layout (time bin, space bin)
    assert raw == [qexact(1.0), 0, qexact(1.0), 0, qexact(1.0), 0]


def test_scripted_regions_change_cross_section(orc):
    # cells [0,1] [1,1.5] [1.5,2] [2,3]; sigma_t 1 left of 1.5, 2 right of it
    p = slab([0, 1.5, 3], [1.0, 2.0], [0.9, 0.5], [0, 1, 2, 3])
    tau0 = -orc.ln(2.0 ** -5)
    raw, d, ev, used = orc.transport_scripted(p, LCG, [2.0 ** -5, 0.99])
    assert used == 2 and d["absorbed"] == 1
    assert [e[0] for e in ev] == [1, 1, 1, 0]
    assert [e[1] for e in ev] == [0, 1, 2, 3]
    tau = tau0 - 1.0 * 1.0
    tau = tau - 1.0 * 0.5
    tau = tau - 2.0 * 0.5
    s = tau / 2.0
    assert ev[3][3] == s
    assert raw == [qexact(1.0), qexact(0.5) + qexact(0.5), qexact(s)]


def test_scripted_float_mode(orc):
    """FP32 flight: position relative to the cell's left edge, every
    distance, position and time operation a single-precision one, widths
    rounded once from doubles; the remaining optical depth stays double and
    is consumed by the exact double product of sigma_t and the float track."""
    p = slab([0, 10], [1.3], [0.5], [0, 3.3, 10])
    raw, d, ev, used = orc.transport_scripted(p, LCG, [2.0 ** -7, 0.25, 0.125, 0.25, 0.75], float_mode=True)
    f = np.float32
    W0, W1, S = f(3.3 - 0.0), f(10.0 - 3.3), f(1.3)
    tau = -orc.ln(2.0 ** -7)                    # double: 4.85..., above 1.3 x 3.3
    s1 = f(f(W0 - f(0)) / f(1))                 # edge of cell 0
    assert f(f(tau) / S) > s1
    tau = tau - float(S) * float(s1)            # exact product, one double subtraction
    s2 = f(f(tau) / S)                          # collision in cell 1, local position s2
    xl = f(f(0) + f(f(1) * s2))
    mu = f(2.0 * 0.125 - 1.0)
    tau = -orc.ln(0.25)
    s3 = f(f(f(0) - xl) / mu)                   # back to the edge at 3.3
    assert f(f(tau) / S) > s3
    tau = tau - float(S) * float(s3)
    s4 = f(f(tau) / S)                          # collision in cell 0, then absorbed
    assert used == 5 and d["absorbed"] == 1
    assert [e[0] for e in ev] == [1, 0, 1, 0] and [e[1] for e in ev] == [0, 1, 1, 0]
    assert [e[3] for e in ev] == [float(s1), float(s2), float(s3), float(s4)]
    assert raw == [qexact(float(s1)) + qexact(float(s4)), qexact(float(s2)) + qexact(float(s3))]


def test_scripted_float_mode_time_local(orc):
    """FP32 time is kept relative to the time bin's start."""
    p = slab([0, 200], [0.3], [1.0], [0, 80, 200], time_edges=[0, 33.3, 100])
    raw, d, ev, used = orc.transport_scripted(p, LCG, [2.0 ** -53], float_mode=True)
    f = np.float32
    assert d["census"] == 1 and used == 1 and [e[0] for e in ev] == [2, 1, 2]
    dt0, dt1, w0 = f(33.3 - 0.0), f(100.0 - 33.3), f(80.0 - 0.0)
    s1 = dt0                                      # end of the first time bin at x = s1
    s2 = f(w0 - s1)                               # the edge at x = 80, local time s2
    s3 = f(dt1 - s2)                              # rest of the second time bin: census
    assert [e[3] for e in ev] == [float(s1), float(s2), float(s3)]
    assert raw == [qexact(float(s1)), 0, qexact(float(s2)), qexact(float(s3))]


# ------------------------------------------------------------ closed forms

def _batch_stats(prob, tally):
    """Per-bin mean track length per history and its standard error from
    the spread of the batch means."""
    nb, nsb = tally.n_batches, tally.n_space_bins * max(tally.n_time_bins, 1)
    n_b = np.array(__import__("oracle").batch_sizes(prob), float)
    per = np.array([[tally.raw[b * nsb + i] / Q56 / n_b[b] for i in range(nsb)] for b in range(nb)])
    return per.mean(0), per.std(0, ddof=1) / math.sqrt(nb)


@pytest.mark.parametrize("float_mode", [False, True])
def test_pure_absorber_closed_form(orc, float_mode):
    S, L, nbins, N = 1.3, 3.0, 6, 200_000
    p = W.homogeneous(L, S, 0.0, nbins, N, n_batches=50)
    t = orc.transport(p, LCG, float_mode=float_mode, threads=8)
    mean, se = _batch_stats(p, t)
    a = np.arange(nbins) * L / nbins
    b = a + L / nbins
    exact = (np.exp(-S * a) - np.exp(-S * b)) / S
    assert np.all(np.abs(mean - exact) < 5 * se + 1e-12)
    pt = math.exp(-S * L)
    assert abs(t.diag["leak_right"] / N - pt) < 5 * math.sqrt(pt * (1 - pt) / N)
    assert t.diag["leak_left"] == 0 and t.diag["absorbed"] + t.diag["leak_right"] == N


def test_time_dependent_pure_absorber(orc):
    S, N = 0.7, 200_000
    te = [0.0, 1.0, 2.5, 4.0, 6.0, 8.0]
    p = slab([0, 10], [S], [0.0], [0, 2, 4, 6, 8, 10], n=N, time_edges=te, n_batches=40)
    t = orc.transport(p, LCG, threads=8)
    mean, se = _batch_stats(p, t)
    exact = []
    for i in range(5):
        for k in range(5):
            lo, hi = max(te[i], 2.0 * k), min(te[i + 1], 2.0 * k + 2.0)
            exact.append((math.exp(-S * lo) - math.exp(-S * hi)) / S if lo < hi else 0.0)
    exact = np.array(exact)
    assert np.all(np.abs(mean - exact) < 5 * se + 1e-12)
    pc = math.exp(-S * 8.0)
    assert abs(t.diag["census"] / N - pc) < 5 * math.sqrt(pc * (1 - pc) / N)


def _H(c, mu, n=200):
    x, w = np.polynomial.legendre.leggauss(n)
    x, w = 0.5 * (x + 1), 0.5 * w
    H = np.ones(n)
    for _ in range(5000):
        Hn = 1.0 / (1.0 - 0.5 * c * x * np.sum(w * H / (x[:, None] + x), axis=1))
        done = np.max(np.abs(Hn - H)) < 1e-14
        H = Hn
        if done:
            break
    return 1.0 / (1.0 - 0.5 * c * mu * np.sum(w * H / (mu + x)))


@pytest.mark.parametrize("c,float_mode", [(0.5, False), (0.9, False), (0.9, True)])
def test_half_space_albedo(orc, c, float_mode):
    N = 100_000
    p = W.homogeneous(60.0, 1.0, c, 4, N)
    t = orc.transport(p, LCG, float_mode=float_mode, threads=8)
    A = 1.0 - math.sqrt(1.0 - c) * _H(c, 1.0)
    assert abs(t.diag["leak_left"] / N - A) < 5 * math.sqrt(A * (1 - A) / N)


def test_albedo_with_identical_regions(orc):
    """Splitting the half-space into regions of the same material changes
    nothing physical (optical depth carries across region edges)."""
    N, c = 100_000, 0.8
    re = np.array([0.0, 0.3, 1.1, 2.0, 7.5, 60.0]) / 2.0
    p = W.SlabProblem(re, np.full(5, 2.0), np.full(5, c), np.linspace(0, 30.0, 9), N)
    t = orc.transport(p, LCG, threads=8)
    A = 1.0 - math.sqrt(1.0 - c) * _H(c, 1.0)
    assert abs(t.diag["leak_left"] / N - A) < 5 * math.sqrt(A * (1 - A) / N)


def test_collision_estimator_identity(orc):
    S, nb, bs = 1.7, 50, 2000
    p = W.homogeneous(5.0, S, 0.9, 10, nb * bs)
    diff = []
    for b in range(nb):
        t = orc.transport(p, LCG, j0=b * bs, j1=(b + 1) * bs)
        diff.append(S * sum(t.raw) / Q56 - t.diag["collisions"])
    diff = np.array(diff) / bs           # per-history (sigma_t * track - collisions), mean 0
    assert abs(diff.mean()) < 5 * diff.std(ddof=1) / math.sqrt(nb)


# ------------------------------------------------------------ exactness properties

@pytest.mark.parametrize("make", [lambda: W.small_slab(), lambda: W.small_slab(W.stride_seeding()),
                                  lambda: W.multi_region(n_histories=3000)])
def test_balance_and_threads(orc, make):
    p = make()
    a = orc.transport(p, LCG, threads=1)
    b = orc.transport(p, LCG, threads=8)
    assert a.raw == b.raw and a.diag == b.diag
    d = a.diag
    assert d["histories"] == p.n_histories
    assert d["leak_left"] + d["leak_right"] + d["absorbed"] + d["census"] == p.n_histories


def test_sharding_and_batches(orc):
    p = W.long_chain(n_histories=6400, n_batches=64)
    whole = orc.transport(p, LCG)
    parts = [orc.transport(p, LCG, j0=a, j1=b) for a, b in ((0, 1000), (1000, 4321), (4321, 6400))]
    assert [sum(v) for v in zip(*(x.raw for x in parts))] == whole.raw
    one = orc.transport(p.with_(n_batches=1), LCG)
    nsb = 200
    assert [sum(whole.raw[b * nsb + i] for b in range(64)) for i in range(nsb)] == one.raw


def _bin_overlap(lo_a, hi_a, lo_b, hi_b):
    lo, hi = max(lo_a, lo_b), min(hi_a, hi_b)
    return (lo, hi) if lo < hi else None


def test_flux_transparent_slab_exact(orc):
    """A nearly transparent time-dependent slab: every particle runs at
    x = t from the left face to the right face, so its track in space bin k
    and time bin i is the overlap of [x_k, x_k+1) with [t_i, t_i+1), the
    same for every history.  The flux of each (batch, time bin, space bin)
    is then exactly that overlap / (dx dt), whatever the batch's size: N is
    not a multiple of the batch count (batch sizes 3, 3, 3, 1), and no
    width is 1."""
    be = [0.0, 0.5, 1.5, 3.0, 4.2]
    te = [0.0, 0.7, 2.0, 3.1, 5.0]
    p = slab([0.0, 2.2, 4.2], [1e-7, 2e-7], [0.0, 0.0], be, n=10, time_edges=te, n_batches=4)
    t = orc.transport(p, LCG)
    assert t.diag["leak_right"] == 10 and t.diag["absorbed"] == 0
    assert orc.batch_sizes(p) == [3, 3, 3, 1]
    fl = orc.flux(p, t).reshape(4, 4, 4)
    for b in range(4):
        for i in range(4):
            for k in range(4):
                ov = _bin_overlap(be[k], be[k + 1], te[i], te[i + 1])
                want = 0.0 if ov is None else (ov[1] - ov[0]) / ((be[k + 1] - be[k]) * (te[i + 1] - te[i]))
                assert fl[b, i, k] == pytest.approx(want, rel=1e-12, abs=0.0), (b, i, k)


def test_flux_time_dependent_absorber_per_batch(orc):
    """Pure absorber (sigma_t = 0.6) at speed 1: the particle is at x = t
    until it is absorbed at a distance S ~ Exp(sigma_t).  Its track in a
    (time bin, space bin) cell whose x = t overlap is [lo, hi) is
    T = min(max(S - lo, 0), hi - lo), with
      E[T]   = e^{-s lo} (1 - e^{-s w}) / s,
      E[T^2] = 2 e^{-s lo} (1/s^2 - e^{-s w} (w/s + 1/s^2)),  w = hi - lo.
    Every batch's flux must lie within 5 standard errors of
    E[T] / (dx dt), with N_b that batch's own history count (N = 40003 in
    6 batches, the last one smaller), dx and dt not 1."""
    S = 0.6
    be = [0.0, 0.8, 2.0, 3.5, 6.0]
    te = [0.0, 0.9, 2.2, 3.0, 4.6, 7.0]
    p = slab([0.0, 6.0], [S], [0.0], be, n=40003, time_edges=te, n_batches=6)
    t = orc.transport(p, LCG, threads=8)
    nb = orc.batch_sizes(p)
    assert nb[-1] < nb[0]
    fl = orc.flux(p, t).reshape(6, 5, 4)
    for i in range(5):
        for k in range(4):
            dxdt = (be[k + 1] - be[k]) * (te[i + 1] - te[i])
            ov = _bin_overlap(be[k], be[k + 1], te[i], te[i + 1])
            if ov is None:
                assert np.all(fl[:, i, k] == 0.0)
                continue
            lo, w = ov[0], ov[1] - ov[0]
            m1 = math.exp(-S * lo) * (1.0 - math.exp(-S * w)) / S
            m2 = 2.0 * math.exp(-S * lo) * (1.0 / S ** 2 - math.exp(-S * w) * (w / S + 1.0 / S ** 2))
            sd = math.sqrt(m2 - m1 * m1)
            for b in range(6):
                se = sd / math.sqrt(nb[b]) / dxdt
                assert abs(fl[b, i, k] - m1 / dxdt) < 5 * se, (b, i, k, fl[b, i, k], m1 / dxdt, se)


def test_stride_exceedance_counted(orc):
    """A tiny stride makes long histories run into the next unit's stream."""
    sd = W.Seeding("stride", 1, 20, 0)
    p = W.small_slab(sd, n_histories=2000)
    t = orc.transport(p, LCG)
    assert t.diag["over_stride"] > 0 and t.diag["max_draws"] > 20
    t2 = orc.transport(W.small_slab(W.stride_seeding(), n_histories=2000), LCG)
    assert t2.diag["over_stride"] == 0
