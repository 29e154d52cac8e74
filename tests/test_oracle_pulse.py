"""Pins of the oracle's pulse problem (a pulse in an infinite multiplying
medium with secondaries seeded on demand, the paper's test problem).

The pins come from outside the oracle's own code: hand-derived families
driven by scripted uniforms, the seed-splitting rule of eq. (5) checked
against the separately pinned hash and LCG primitives, exact particle and
draw balances, and closed forms of the expected collision counts (pure
absorber, critical pure scatterer, supercritical growth e^{(c nu - 1) t}),
and the flux normalisation against the pure absorber's uncollided flux
(sigma_t, window and time-bin widths not 1, several batches)."""
import math

import numpy as np
import pytest
from scipy.special import exp1

import workloads as W

LCG = W.Lcg()
LN2 = 0.6931471805599453   # the double nearest ln 2 (ln(0.5) = -LN2 exactly in the oracle)
MASK = (1 << 63) - 1


def prob(**kw):
    base = dict(sigma_t=2.0, scatter=0.5, nu=1.5, x_lo=-1.0, x_hi=1.0,
                time_edges=np.array([0.0, 1.0, 2.0, 4.0]), n_batches=1, per_batch=1,
                seeding=W.stride_seeding())
    base.update(kw)
    return W.PulseProblem(**base)


def test_scripted_family_by_hand(orc):
    """Source: mu = 2(0.75) - 1 = 0.5, tau = ln 2, s0 = ln2/2; it collides at
    x = 0.5 s0, t = s0 (bin 0, scored) and scatters (0.25 < 0.5) into
    n = 1 + (0.25 < 0.5) = 2.  First child: mu = 1, tau = -ln 1 = 0, collides
    where it stands (bin 0), absorbed (0.9).  Second child: mu = -0.75,
    tau = ln 4, s = ln 2: collides at t = s0 + ln2 (bin 1),
    x = 0.5 s0 - 0.75 ln2 (inside [-1, 1]), absorbed (0.5 is not < 0.5)."""
    u = [0.75, 0.5, 0.25, 0.25,
         1.0, 1.0, 0.9,
         0.125, 0.25, 0.5]
    counts, d, used = orc.pulse_scripted(prob(), LCG, u)
    s0 = LN2 / 2.0
    assert 1.0 <= s0 + LN2 < 2.0 and -1.0 <= 0.5 * s0 - 0.75 * LN2 <= 1.0
    assert counts == [2, 1, 0]
    assert used == 10
    assert d == dict(sources=1, collisions=3, tallied=3, scatters=1, absorbed=2, census=0,
                     secondaries=2, draws=10, max_draws=10, over_stride=0)


def test_scripted_depth_first(orc):
    """Source (mu = 1) collides at t = s0 = ln2/2 and scatters into two; its
    first child collides at t = ln2 and scatters into two again.  Depth
    first, the next three particles of the script are the two grandchildren
    (starting at t = ln2) and then the source's second child (t = s0):
      3rd: tau = ln 16, s = 2 ln2 -> t = 3 ln2 (bin 2), absorbed
      4th: tau = 53 ln2 -> census
      5th: tau = ln 2, s = s0 -> t = ln2 (bin 0), absorbed.
    Breadth first (second child before the grandchildren) the same script
    would give collisions at t = s0 + 2 ln2 and t = ln2 + s0, both in bin 1."""
    u = [1.0, 0.5, 0.25, 0.25,
         1.0, 0.5, 0.25, 0.25,
         1.0, 0.0625, 0.9,
         1.0, 2.0 ** -53,
         1.0, 0.5, 0.9]
    wide = prob(x_lo=-10.0, x_hi=10.0)
    counts, d, used = orc.pulse_scripted(wide, LCG, u)
    assert 2.0 <= 3 * LN2 < 4.0
    assert counts == [3, 0, 1]
    assert used == 16
    assert d == dict(sources=1, collisions=4, tallied=4, scatters=2, absorbed=2, census=1,
                     secondaries=4, draws=16, max_draws=16, over_stride=0)
    # mu = 1 puts every particle at x = t: with x in [-1, 1] the collision at 3 ln2 is outside
    counts, _, _ = orc.pulse_scripted(prob(), LCG, u)
    assert counts == [3, 0, 0]


def test_scripted_edges(orc):
    """A collision exactly on a time edge goes to the later bin; x exactly on
    x_hi is scored; a flight ending exactly at the census time reaches the
    census; nu = 0.5 with u2 >= 0.5 ends the family with no successor."""
    s = LN2 / 1.0
    p = prob(sigma_t=1.0, nu=0.5, time_edges=np.array([0.0, s, 4.0]), x_hi=0.5 * s)
    counts, d, _ = orc.pulse_scripted(p, LCG, [0.75, 0.5, 0.25, 0.5])
    assert counts == [0, 1] and d["scatters"] == 1 and d["secondaries"] == 0
    assert d["tallied"] == 1
    p2 = prob(sigma_t=1.0, time_edges=np.array([0.0, 0.5, s]))
    counts, d, used = orc.pulse_scripted(p2, LCG, [0.75, 0.5])
    assert counts == [0, 0] and d["census"] == 1 and d["collisions"] == 0 and used == 2
    # tau = 0 collides where it stands: a source with t_edges[0] > 0 is not scored
    p3 = prob(time_edges=np.array([0.5, 1.0, 2.0]))
    counts, d, _ = orc.pulse_scripted(p3, LCG, [1.0, 1.0, 0.9])
    assert counts == [0, 0] and d["collisions"] == 1 and d["tallied"] == 0


def test_child_seed_rule_hash(orc):
    """Eq. (5): the k-th particle emerging from a scattering starts at
    hash(k, X_p) mod 2^63, X_p the parent's state after its draws; every
    particle's stream is its own (2 draws at census, 3 when absorbed, 4 when
    it scatters) and the source starts at hash(i+1, hash(B+1, s))."""
    p = W.pulse(W.hash_seeding(), n_batches=4, per_batch=50, first_batch=7)
    for b, i in ((0, 0), (3, 17), (2, 49)):
        _, d, recs = orc.pulse_trace(p, LCG, b, i)
        assert recs[0][0] == orc.hash64(i + 1, orc.hash64(7 + b + 1, 1)) & MASK
        expected_children = []
        for start, end, _, _, n_out, draws in recs:
            x = start
            for _ in range(draws):
                x = orc.lcg_next(x, LCG.g, LCG.c, LCG.m)
            assert x == end
            if n_out:
                assert draws == 4
            else:
                assert draws in (2, 3)
            expected_children += [orc.hash64(k, end) & MASK for k in range(1, n_out + 1)]
        starts = sorted(r[0] for r in recs[1:])
        assert starts == sorted(expected_children)
        assert d["sources"] == 1 and d["secondaries"] == len(recs) - 1
        assert d["max_draws"] <= 4


def test_stride_family_one_stream(orc):
    """Stride seeding: source i of batch B starts at X_{Q (B per_batch + i)}
    and the whole family consumes that one stream in processing order."""
    p = W.pulse(W.stride_seeding(), n_batches=3, per_batch=40, first_batch=2)
    b, i = 1, 33
    _, d, recs = orc.pulse_trace(p, LCG, b, i)
    assert recs[0][0] == orc.skip(1, 152917 * ((2 + b) * 40 + i), LCG.g, LCG.c, LCG.m)
    for prev, cur in zip(recs, recs[1:]):
        assert cur[0] == prev[1]
    assert d["draws"] == sum(r[5] for r in recs) == d["max_draws"]


@pytest.mark.parametrize("kind", ["hash", "stride"])
def test_exact_balances(orc, kind):
    sd = W.hash_seeding() if kind == "hash" else W.stride_seeding()
    p = W.pulse(sd, n_batches=40, per_batch=200)
    r = orc.pulse(p, LCG, threads=4)
    d = r.diag
    particles = d["sources"] + d["secondaries"]
    assert d["sources"] == 8000
    assert particles == d["absorbed"] + d["census"] + d["scatters"]
    assert d["collisions"] == d["absorbed"] + d["scatters"]
    assert d["draws"] == 2 * particles + d["collisions"] + d["scatters"]
    assert int(r.counts.sum()) == d["tallied"] <= d["collisions"]


def test_threads_batches_and_offsets(orc):
    p = W.pulse(W.hash_seeding(), n_batches=12, per_batch=100)
    a = orc.pulse(p, LCG, threads=1)
    b = orc.pulse(p, LCG, threads=5)
    assert np.array_equal(a.counts, b.counts) and a.diag == b.diag
    lo = orc.pulse(p, LCG, 0, 7)
    hi = orc.pulse(p, LCG, 7, 12)
    assert np.array_equal(lo.counts + hi.counts, a.counts)
    sub = orc.pulse(p.with_(n_batches=5, first_batch=7), LCG)
    assert np.array_equal(sub.counts, a.counts[7:])


def _batch_mean_and_se(counts, per_batch):
    m = counts.astype(np.float64) / per_batch
    return m.mean(axis=0), m.std(axis=0, ddof=1) / math.sqrt(m.shape[0])


def test_pure_absorber_closed_form(orc):
    """c = 0: each source collides once, at distance s ~ Exp(sigma_t) in
    direction mu ~ U[-1, 1]; with sigma_t = 1 and x in [-1, 1] the expected
    count per source in [a, b) is the integral of e^{-s} min(1, 1/s):
    1 - e^{-1} on [0, 1) and E1(a) - E1(b) beyond."""
    p = W.PulseProblem(scatter=0.0, time_edges=np.array([0.0, 1.0, 2.0, 3.0, 5.0]),
                       n_batches=200, per_batch=2000, seeding=W.hash_seeding())
    r = orc.pulse(p, LCG, threads=8)
    n = p.n_sources
    expect = np.array([1.0 - math.exp(-1.0), exp1(1.0) - exp1(2.0), exp1(2.0) - exp1(3.0),
                       exp1(3.0) - exp1(5.0)])
    got = r.counts.sum(axis=0) / n
    se = np.sqrt(expect * (1 - expect) / n)
    assert np.all(np.abs(got - expect) < 5 * se), (got, expect)
    assert r.diag["collisions"] + r.diag["census"] == n and r.diag["scatters"] == 0


def test_critical_pure_scatterer_poisson(orc):
    """c = 1, nu = 1: exactly one particle is alive at any time, its
    collisions form a Poisson process of rate sigma_t, so the count over all
    x in a time bin of width w has mean and variance sigma_t w per source."""
    p = W.PulseProblem(sigma_t=1.5, scatter=1.0, nu=1.0, x_lo=-1e300, x_hi=1e300,
                       time_edges=np.array([0.0, 0.5, 2.0, 4.0]), n_batches=100, per_batch=1000,
                       seeding=W.stride_seeding())
    r = orc.pulse(p, LCG, threads=8)
    n = p.n_sources
    w = np.diff(p.time_edges)
    got = r.counts.sum(axis=0) / n
    assert np.all(np.abs(got - 1.5 * w) < 5 * np.sqrt(1.5 * w / n)), got
    assert r.diag["secondaries"] == r.diag["scatters"] == r.diag["collisions"]
    assert r.diag["census"] == n


@pytest.mark.parametrize("kind", ["hash", "stride"])
def test_supercritical_growth_closed_form(orc, kind):
    """c nu = 1.1, sigma_t = 1, v = 1: the expected population is
    e^{0.1 t}, so the expected number of collisions (all x) in [a, b) per
    source is 10 (e^{0.1 b} - e^{0.1 a}).  Standard errors from batch means."""
    sd = W.hash_seeding() if kind == "hash" else W.stride_seeding()
    p = W.pulse(sd, n_batches=400, per_batch=250).with_(x_lo=-1e300, x_hi=1e300)
    r = orc.pulse(p, LCG, threads=8)
    t = p.time_edges
    expect = 10.0 * (np.exp(0.1 * t[1:]) - np.exp(0.1 * t[:-1]))
    mean, se = _batch_mean_and_se(r.counts, p.per_batch)
    z = (mean - expect) / se
    assert np.all(np.abs(z) < 5.0), z


def test_hash_and_stride_agree_in_distribution(orc):
    """The center-flux means of the two seedings agree within their errors."""
    ph = W.pulse(W.hash_seeding(), n_batches=200, per_batch=500)
    ps = ph.with_(seeding=W.stride_seeding())
    mh, sh = _batch_mean_and_se(orc.pulse(ph, LCG, threads=8).counts, 500)
    ms, ss = _batch_mean_and_se(orc.pulse(ps, LCG, threads=8).counts, 500)
    z = (mh - ms) / np.sqrt(sh ** 2 + ss ** 2)
    assert np.all(np.abs(z) < 5.0), z


def _absorber_hit_prob(sig, x_lo, x_hi, a, b):
    """P(one source of a pure absorber collides at a time in [a, b) inside
    [x_lo, x_hi]), x_lo < 0 < x_hi: the collision is at distance s with
    density sig e^{-sig s}, at time s (speed 1) and position mu s with
    mu ~ U[-1, 1], so P(x_lo <= mu s <= x_hi) = (min(1, x_hi/s) -
    max(-1, x_lo/s)) / 2."""
    from scipy.integrate import quad

    def f(s):
        g = 1.0 if s == 0.0 else 0.5 * (min(1.0, x_hi / s) - max(-1.0, x_lo / s))
        return sig * math.exp(-sig * s) * g
    brk = [v for v in (abs(x_lo), x_hi) if a < v < b]
    return quad(f, a, b, points=brk or None, epsabs=1e-14, epsrel=1e-12)[0]


def test_flux_pure_absorber_closed_form(orc):
    """The flux normalisation against physics: for a pure absorber the
    scalar flux is the uncollided flux e^{-sig t} / (2 t) for |x| < t, and
    the collision estimator count / (sig N_b (x_hi - x_lo) dt) must
    estimate its space-time average P_hit / (sig (x_hi - x_lo) dt) in every
    batch (within 5 binomial standard errors), with sigma_t, the window and
    the time-bin widths all different from 1 and several batches."""
    sig, x_lo, x_hi = 1.7, -0.5, 1.2
    te = np.array([0.0, 0.4, 1.0, 2.5, 4.0])
    p = W.PulseProblem(sigma_t=sig, scatter=0.0, x_lo=x_lo, x_hi=x_hi, time_edges=te, n_batches=5,
                       per_batch=20000, seeding=W.hash_seeding())
    r = orc.pulse(p, LCG, threads=8)
    f = orc.pulse_flux(p, LCG, r.counts)
    for k in range(len(te) - 1):
        ph = _absorber_hit_prob(sig, x_lo, x_hi, te[k], te[k + 1])
        den = sig * (x_hi - x_lo) * (te[k + 1] - te[k])
        se = math.sqrt(ph * (1.0 - ph) / p.per_batch) / den
        for b in range(p.n_batches):
            assert abs(f[b, k] - ph / den) < 5 * se, (b, k, f[b, k], ph / den, se)
