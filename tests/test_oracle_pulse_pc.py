"""Pins of the oracle's population control for the pulse problem: a census
every K time bins, after which each batch holds M particles on average.  The
decisions are one-off hashed values of a per-phase seed (Sec. "Hierarchical
Seed Splitting"), and the copies are seeded like eq. (5)'s secondaries.

The pins come from outside the oracle's code:
* a hand-derived family up to the first census (census point and direction);
* the copy rule re-derived with exact rational arithmetic from the pinned
  hash primitive;
* exact particle and draw balances;
* the supercritical closed form e^{0.1 t}, which the weighted estimate must
  still meet;
* agreement in distribution with the uncontrolled problem;
* the weighted flux normalisation against the pure absorber's closed form
  (sigma_t, window and time-bin widths not 1, a census that changes the
  population, so a missing weight, sigma_t or dt fails)."""
import math
from fractions import Fraction

import numpy as np
import pytest

import workloads as W

LCG = W.Lcg()
MASK = (1 << 63) - 1


def scripted_prob(**kw):
    base = dict(sigma_t=1.0, scatter=0.4, nu=2.75, x_lo=-1.0, x_hi=1.0,
                time_edges=np.arange(11, dtype=np.float64), n_batches=1, per_batch=1,
                seeding=W.stride_seeding(), census_every=5, pc_target=1)
    base.update(kw)
    return W.PulseProblem(**base)


def test_scripted_census_by_hand(orc):
    """A source flying past the first census (T[5] = 5) stops at
    x + mu (5 - t) with its direction: mu = 2(0.75) - 1 = 0.5, so x = 2.5."""
    p = scripted_prob()
    cnt, d, used, arr = orc.pulse_pc_scripted(p, LCG, [0.75, math.exp(-6.0)])
    assert used == 2 and arr == [(2.5, 0.5)]
    assert sum(cnt) == 0
    assert d["census"] == 1 and d["collisions"] == 0 and d["draws"] == 2


def test_scripted_census_family_by_hand(orc):
    """Source: mu = 0.5, flight ~1.5 -> collision at x ~ 0.75, t ~ 1.5 (bin 1,
    scored), u1 = 0.1 scatters, u2 = 0.5 < 0.75 gives 3 particles.  Depth
    first: child 1 (mu = -0.5, flight ~10) reaches the census at
    0.75 - 0.5 (5 - 1.5) ~ -1.0; child 2 (mu = 1, flight ~2) collides at
    x ~ 2.75, unscored, and u1 = 0.9 absorbs it; child 3 (mu = 0, flight
    ~20) reaches the census where it started, x ~ 0.75."""
    p = scripted_prob()
    u = [0.75, math.exp(-1.5), 0.1, 0.5,
         0.25, math.exp(-10.0),
         1.0, math.exp(-2.0), 0.9,
         0.5, math.exp(-20.0)]
    cnt, d, used, arr = orc.pulse_pc_scripted(p, LCG, u)
    assert used == len(u)
    assert cnt == [0, 1, 0, 0, 0, 0, 0, 0, 0, 0]
    assert len(arr) == 2
    assert abs(arr[0][0] - (-1.0)) < 1e-12 and arr[0][1] == -0.5
    assert abs(arr[1][0] - 0.75) < 1e-12 and arr[1][1] == 0.0
    assert d == {"sources": 1, "collisions": 2, "tallied": 1, "scatters": 1, "absorbed": 1, "census": 2,
                 "secondaries": 3, "draws": 11, "max_draws": 11, "over_stride": 0}


def pc_prob(**kw):
    base = dict(n_batches=6, per_batch=120, census_every=4, target=150)
    base.update(kw)
    return W.pulse_pc(**base)


def copies_by_definition(arrivals, M, phi):
    """Copies of each arrival X at a census of N = len(arrivals) particles,
    from the definition: q = floor(M/N), r = M mod N, one more copy when the
    one-off value U(hash(X, phi)) is below r/N (exact rationals); copy k
    starts at hash(k, X)."""
    N = len(arrivals)
    q, r = divmod(M, N)
    out = []
    for X in arrivals:
        S = W_hash(X, phi) & MASK
        u = Fraction((S >> 10) + 1, 1 << 53)
        n = q + (1 if u < Fraction(r, N) else 0)
        out += [W_hash(k, X) & MASK for k in range(1, n + 1)]
    return out


W_hash = None


@pytest.fixture(autouse=True)
def _hash(orc):
    global W_hash
    W_hash = orc.hash64


@pytest.mark.parametrize("target", [150, 1, 1000])
def test_copies_follow_the_one_off_rule(orc, target):
    """Copy numbers and copy seeds at each census follow the one-off rule:
    the phase seed is hash(c+1, hash(B+1, pc_seed)), each arrival's state its
    key; the per-batch populations the run reports agree."""
    p = pc_prob(target=target, n_batches=3).with_(first_batch=5)
    run = orc.pulse_pc(p, LCG)
    nc = orc.pc_n_census(p)
    assert nc == 4
    for b in range(p.n_batches):
        for c in range(nc):
            arr, cop = orc.pulse_pc_census(p, LCG, b, c)
            assert run.pop[b, c, 0] == len(arr)
            assert run.pop[b, c, 1] == len(cop)
            if not arr:
                assert not cop
                continue
            phi = orc.hash64(c + 1, orc.hash64(5 + b + 1, p.pc_seed))
            assert cop == copies_by_definition(arr, target, phi)


def test_population_bounds_and_mean(orc):
    """q N <= copies <= (q + 1) N at every census (q = floor(M/N)), and the
    copies average M (binomial spread of the r extra copies)."""
    p = pc_prob(n_batches=300, per_batch=60, target=75)
    r = orc.pulse_pc(p, LCG, threads=8)
    N = r.pop[:, :, 0].astype(np.int64)
    K = r.pop[:, :, 1].astype(np.int64)
    live = N > 0
    q = np.where(live, 75 // np.maximum(N, 1), 0)
    assert np.all(K[live] >= (q * N)[live]) and np.all(K[live] <= ((q + 1) * N)[live])
    assert np.all(K[~live] == 0)
    rr = np.where(live, 75 % np.maximum(N, 1), 0)
    var = (rr * (1.0 - rr / np.maximum(N, 1)))[live].sum()
    z = (K[live].sum() - 75 * live.sum()) / math.sqrt(var)
    assert abs(z) < 5.0, z


def test_pc_balances(orc):
    """Every particle (source, secondary or census copy) ends once: absorbed,
    at a census or at a scattering; sources and secondaries draw a direction
    and a flight, copies only a flight."""
    p = pc_prob(n_batches=20, per_batch=200)
    r = orc.pulse_pc(p, LCG, threads=4)
    d = r.diag
    copies = int(r.pop[:, :, 1].sum())
    assert d["sources"] + d["secondaries"] + copies == d["absorbed"] + d["census"] + d["scatters"]
    assert d["draws"] == 2 * (d["sources"] + d["secondaries"]) + copies + d["collisions"] + d["scatters"]
    assert int(r.counts.sum()) == d["tallied"]


def test_no_census_point_is_the_plain_problem(orc):
    """With no census before the last edge the run is the plain problem."""
    p = pc_prob(n_batches=5, census_every=20)
    assert orc.pc_n_census(p) == 0
    r = orc.pulse_pc(p, LCG)
    ref = orc.pulse(p, LCG)
    assert np.array_equal(r.counts, ref.counts) and r.diag == ref.diag
    assert np.array_equal(orc.pulse_pc_flux(p, LCG, r.counts, r.pop), orc.pulse_flux(p, LCG, ref.counts))


def test_threads_batches_and_offsets(orc):
    p = pc_prob(n_batches=8, per_batch=80)
    whole = orc.pulse_pc(p, LCG)
    split = orc.pulse_pc(p, LCG, threads=3)
    assert np.array_equal(whole.counts, split.counts) and whole.diag == split.diag
    assert np.array_equal(whole.pop, split.pop)
    part = orc.pulse_pc(p, LCG, 2, 5)
    assert np.array_equal(part.counts[2:5], whole.counts[2:5]) and not part.counts[:2].any()
    assert np.array_equal(part.pop[2:5], whole.pop[2:5])
    shifted = orc.pulse_pc(p.with_(n_batches=3, first_batch=5), LCG)
    assert np.array_equal(shifted.counts, whole.counts[5:8]) and np.array_equal(shifted.pop, whole.pop[5:8])


def test_extinct_batch(orc):
    """A pure absorber with a late first census: batches die out; a batch
    with no arrivals has no copies and scores nothing after the census."""
    p = pc_prob(n_batches=50, per_batch=1).with_(scatter=0.0)
    r = orc.pulse_pc(p, LCG)
    dead = r.pop[:, 0, 0] == 0
    assert dead.any()
    assert not r.pop[dead].any()
    assert not r.counts[dead][:, 4:].any()


def _weighted_per_source(orc, p, r):
    """count x epoch weight / per_batch from the flux: flux x sigma_t dx dt."""
    f = orc.pulse_pc_flux(p, LCG, r.counts, r.pop)
    dt = np.diff(p.time_edges)
    return f * p.sigma_t * (p.x_hi - p.x_lo) * dt


def test_weighted_growth_closed_form(orc):
    """c nu = 1.1, sigma_t = 1, v = 1: the expected collisions (all x) in
    [a, b) per source are 10 (e^{0.1 b} - e^{0.1 a}) with or without
    population control; the controlled run keeps each batch near M particles
    and carries the growth in the epoch weights."""
    p = pc_prob(n_batches=400, per_batch=250, target=250, census_every=4).with_(x_lo=-1e300, x_hi=1e300)
    r = orc.pulse_pc(p, LCG, threads=8)
    m = _weighted_per_source(orc, p, r)
    mean, se = m.mean(axis=0), m.std(axis=0, ddof=1) / math.sqrt(m.shape[0])
    t = p.time_edges
    expect = 10.0 * (np.exp(0.1 * t[1:]) - np.exp(0.1 * t[:-1]))
    z = (mean - expect) / se
    assert np.all(np.abs(z) < 5.0), z
    # the population is controlled: copies stay near M while arrivals grow
    assert abs(r.pop[:, :, 1].mean() - 250) < 5


def test_center_flux_agrees_with_plain(orc):
    """The center-interval flux with population control agrees in
    distribution with the uncontrolled problem's."""
    p = pc_prob(n_batches=300, per_batch=300, target=300, census_every=5)
    r = orc.pulse_pc(p, LCG, threads=8)
    fp = orc.pulse_pc_flux(p, LCG, r.counts, r.pop)
    ref = orc.pulse(p, LCG, threads=8)
    fr = orc.pulse_flux(p, LCG, ref.counts)
    z = (fp.mean(0) - fr.mean(0)) / np.sqrt(fp.var(0, ddof=1) / fp.shape[0] + fr.var(0, ddof=1) / fr.shape[0])
    assert np.all(np.abs(z) < 5.0), z


def test_weighted_flux_pure_absorber_closed_form(orc):
    """Population control must not bias the flux: a pure absorber
    (sigma_t = 1.7) with a census at t = 1.0 that brings each batch's ~180
    survivors back to 300 (weight ~0.6 afterwards).  Each time bin's mean
    flux over the batches meets the uncollided closed form
    P_hit / (sigma_t (x_hi - x_lo) dt) within 5 standard errors of the
    batch means."""
    from test_oracle_pulse import _absorber_hit_prob
    sig, x_lo, x_hi = 1.7, -0.5, 1.2
    te = np.array([0.0, 0.4, 1.0, 2.5, 4.0])
    p = W.PulseProblem(sigma_t=sig, scatter=0.0, x_lo=x_lo, x_hi=x_hi, time_edges=te, n_batches=200,
                       per_batch=1000, seeding=W.hash_seeding(), census_every=2, pc_target=300)
    r = orc.pulse_pc(p, LCG, threads=8)
    assert r.pop.shape == (200, 1, 2) and abs(r.pop[:, 0, 1].mean() - 300) < 5
    assert abs(r.pop[:, 0, 0].mean() - 1000 * math.exp(-sig)) < 5
    f = orc.pulse_pc_flux(p, LCG, r.counts, r.pop)
    mean, se = f.mean(axis=0), f.std(axis=0, ddof=1) / math.sqrt(f.shape[0])
    for k in range(len(te) - 1):
        want = _absorber_hit_prob(sig, x_lo, x_hi, te[k], te[k + 1]) / (sig * (x_hi - x_lo) * (te[k + 1] - te[k]))
        assert abs(mean[k] - want) < 5 * se[k], (k, mean[k], want, se[k])


def test_rejects_stride_and_missing_target(orc):
    p = pc_prob(n_batches=1)
    with pytest.raises(ValueError):
        orc.pulse_pc(p.with_(seeding=W.stride_seeding()), LCG)
    with pytest.raises(ValueError):
        orc.pulse_pc(p.with_(pc_target=0), LCG)
