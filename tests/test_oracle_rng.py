"""Pins of the oracle's RNG half against what the paper and number theory fix.

* eq. (1) LCG: first step in closed form; Hull-Dobell full period 2^m checked
  by brute force at m = 16, and a multiplier that breaks the condition gives
  a shorter period; the low k bits of an LCG modulo 2^m form an LCG modulo 2^k.
* eq. (2) skip-ahead: equals k brute-force steps; semigroup law; the period
  2^63 at m = 63 (skip(2^63) = id, skip(2^62) != id).
* stride allocation (Sec. "Parallel LCG with Seed Striding"): disjoint and
  covering when N Q = 2^m (brute force at m = 16), overlapping once N Q > 2^m;
  at m = 63 stream k's Q-th output is stream k+1's start state.
* Listing 1 hash: hash(0, 8M) = 0 by hand from the definition; an
  independent inverse (multiplication by M^-1 mod 2^64 and the xorshift
  involution) recovers k from hash(k, s); avalanche statistics.
* eqs. (3), (4): sharding and group-key composition of hash seeds.
* logarithm: within 1.25 ulp of mpmath; exact at 1; powers of two.
* u128 -> double: equals Python's correctly rounded int -> float.
* uniforms: every stream's outputs recomputed with Python integers; range
  and first two moments.
"""
import math
import random

import mpmath
import numpy as np
import pytest

import workloads as W

G = W.G_MCNP
M = 0xC6A4A7935BD1E995
MASK64 = (1 << 64) - 1
MASK63 = (1 << 63) - 1


# ------------------------------------------------------------ eq. (1)

def test_first_step_closed_form(orc):
    # X_1 = g X_0 + c mod 2^63 from X_0 = 1 (stride base seed of the configs)
    assert orc.lcg_next(1, G, 1, 63) == 2806196910506780710
    assert orc.lcg_next(0, G, 1, 63) == 1
    # reduction modulo 2^63 of a product that overflows 64 bits
    x = MASK63
    assert orc.lcg_next(x, G, 1, 63) == (G * x + 1) % (1 << 63)


def _period(orc, g, c, m, x0=0):
    x, n = x0, 0
    seen = set()
    while True:
        x = orc.lcg_next(x, g, c, m)
        n += 1
        if x == x0:
            return n, len(seen)
        seen.add(x)
        if n > (1 << m) + 1:
            return None, len(seen)


def test_full_period_m16_brute_force(orc):
    """Hull-Dobell: c odd and g = 1 (mod 4) give period exactly 2^m."""
    g16 = G % (1 << 16)
    assert g16 % 4 == 1
    n, distinct = _period(orc, g16, 1, 16)
    assert n == 1 << 16 and distinct == (1 << 16) - 1   # every other state before X_0 returns
    # a multiplier with g = 3 (mod 4) violates the condition: shorter period
    n_bad, _ = _period(orc, (g16 + 2) % (1 << 16), 1, 16)
    assert n_bad < (1 << 16)
    # an even increment violates it too
    n_even, _ = _period(orc, g16, 2, 16)
    assert n_even is None or n_even < (1 << 16)


def test_low_bits_form_smaller_lcg(orc):
    rnd = random.Random(3)
    for _ in range(200):
        x = rnd.getrandbits(63)
        for k in (1, 7, 31, 52):
            assert orc.lcg_next(x, G, 1, 63) % (1 << k) == orc.lcg_next(x % (1 << k), G % (1 << k), 1, k)


# ------------------------------------------------------------ eq. (2)

def test_skip_equals_brute_force(orc):
    x0 = 1
    x = x0
    checkpoints = {0, 1, 2, 3, 5, 8, 64, 1000, 152917, 300000}
    for k in range(300001):
        if k in checkpoints:
            assert orc.skip(x0, k, G, 1, 63) == x, k
        x = orc.lcg_next(x, G, 1, 63)
    # another start state and a generic multiplier / increment at m = 64
    rnd = random.Random(5)
    for _ in range(5):
        g, c, x0, k = rnd.getrandbits(64) | 1, rnd.getrandbits(64), rnd.getrandbits(64), rnd.randrange(5000)
        y = x0
        for _ in range(k):
            y = orc.lcg_next(y, g, c, 64)
        assert orc.skip(x0, k, g, c, 64) == y


def test_skip_semigroup(orc):
    rnd = random.Random(11)
    for _ in range(300):
        a, b = rnd.getrandbits(63), rnd.getrandbits(63)
        x0 = rnd.getrandbits(63)
        assert orc.skip(orc.skip(x0, a, G, 1, 63), b, G, 1, 63) == orc.skip(x0, a + b, G, 1, 63)


def test_period_2_63(orc):
    rnd = random.Random(13)
    for _ in range(20):
        x0 = rnd.getrandbits(63)
        assert orc.skip(x0, 1 << 63, G, 1, 63) == x0
        assert orc.skip(x0, 1 << 62, G, 1, 63) != x0
        assert orc.skip(x0, 3 << 61, G, 1, 63) != x0


def test_printed_eq2_is_x0_equal_one_case(orc):
    # eq. (2) as printed: X_k = prod (g^{2^j})^{k_j} + c(1 + ... + g^{k-1}); with X_0 = 1
    for k in (1, 2, 17, 152917, 10 ** 12):
        Gk, Ck = orc.skip_coeffs(k, G, 1, 63)
        assert Gk == pow(G, k, 1 << 63)            # the product of squarings is g^k
        assert orc.skip(1, k, G, 1, 63) == (Gk + Ck) % (1 << 63)


# ------------------------------------------------------------ stride allocation

def test_stride_partition_m16(orc):
    g16 = G % (1 << 16)
    lcg = W.Lcg(g16, 1, 16)
    for Q, N in ((1 << 10, 64), (1000, 65)):
        seen = set()
        total = 0
        for k in range(N):
            x = orc.stream_start(lcg, W.Seeding("stride", 0, Q, 0), k)
            for _ in range(Q):
                seen.add(x)
                x = orc.lcg_next(x, g16, 1, 16)
                total += 1
        assert len(seen) == total          # N Q <= 2^16: no state repeats
        if N * Q == 1 << 16:
            assert len(seen) == 1 << 16    # and the strides cover the cycle
    # N Q > 2^16: the allocations wrap and collide
    Q, N = 1000, 70
    seen, total = set(), 0
    for k in range(N):
        x = orc.stream_start(lcg, W.Seeding("stride", 0, Q, 0), k)
        for _ in range(Q):
            seen.add(x)
            x = orc.lcg_next(x, g16, 1, 16)
            total += 1
    assert len(seen) < total


def test_stride_adjacency_m63(orc):
    lcg = W.Lcg()
    Q = W.STRIDE_Q
    for k in (0, 1, 1000, (1 << 26) - 2):
        sd = W.stride_seeding()
        x = orc.stream_start(lcg, sd, k)
        nxt = orc.stream_start(lcg, sd, k + 1)
        y = orc.skip(x, Q, G, 1, 63)
        assert y == nxt                                  # Q-th output = next stream's start
        assert orc.lcg_next(y, G, 1, 63) == orc.lcg_next(nxt, G, 1, 63)
    assert orc.stream_start(lcg, W.stride_seeding(), 0) == 1   # unit 0 gets X_0


# ------------------------------------------------------------ Listing 1

def _inv_subhash(v):
    y = v ^ (v >> 47)          # y -> y ^ (y >> 47) is its own inverse for shifts >= 32
    return (y * pow(M, -1, 1 << 64)) & MASK64


def test_hash_special_cases(orc):
    assert (8 * M) & MASK64 == 0x35253C9ADE8F4CA8
    assert orc.subhash(0) == 0
    # s = 8M makes s ^ 8M = 0, so seed_hash = 0, and k = 0 gives subhash(0) = 0
    assert orc.hash64(0, (8 * M) & MASK64) == 0
    assert orc.hash64(1, (8 * M) & MASK64) != 0


def test_hash_inverse_round_trip(orc):
    rnd = random.Random(17)
    minv = pow(M, -1, 1 << 64)
    for _ in range(20000):
        k, s = rnd.getrandbits(64), rnd.getrandbits(64)
        h = orc.hash64(k, s)
        sh = _inv_subhash(orc.hash64(0, s))           # seed part, from hash(0, s)
        mixed = _inv_subhash(h) ^ sh                  # = subhash(k) * M
        assert _inv_subhash((mixed * minv) & MASK64) == k


def test_hash_injective_in_key(orc):
    s = 1
    vals = {orc.hash64(k, s) for k in range(1, 200001)}
    assert len(vals) == 200000


def test_hash_avalanche(orc):
    rnd = random.Random(19)
    flips_k, flips_s, n = 0, 0, 0
    for _ in range(400):
        k, s = rnd.getrandbits(64), rnd.getrandbits(64)
        h = orc.hash64(k, s)
        for b in range(0, 64, 3):
            flips_k += bin(h ^ orc.hash64(k ^ (1 << b), s)).count("1")
            flips_s += bin(h ^ orc.hash64(k, s ^ (1 << b))).count("1")
            n += 1
    # a well-mixed 64-bit output flips 32 bits on average (sd 4 per trial)
    assert abs(flips_k / n - 32) < 0.5
    assert abs(flips_s / n - 32) < 0.5


# ------------------------------------------------------------ eqs. (3), (4)

def test_hash_seeding_keys_and_groups(orc):
    lcg = W.Lcg()
    # eq. (3): S_k = hash(k, s), k = 1..N, reduced modulo 2^63
    for i in (0, 1, 99):
        assert orc.stream_start(lcg, W.hash_seeding(), i) == orc.hash64(i + 1, 1) & MASK63
    # sharding: stream i of a set starting at first_index f is global stream f + i
    for f, i in ((10, 5), (1 << 33, 7)):
        assert orc.stream_start(lcg, W.hash_seeding(first_index=f), i) == \
            orc.stream_start(lcg, W.hash_seeding(), f + i)
    # eq. (4): S_{p,j} = hash(j, hash(p, s)): a group key equals a flat set whose seed is hash(p, s)
    for p in (1, 2, 512):
        parent = orc.hash64(p, 1)
        for j in (0, 3):
            assert orc.stream_start(lcg, W.hash_seeding(group_key=p), j) == \
                orc.stream_start(lcg, W.hash_seeding(base=parent), j)


def test_init_streams_matches_stream_start(orc):
    lcg = W.Lcg()
    for sd in (W.hash_seeding(first_index=3), W.stride_seeding(first_index=1000)):
        arr = orc.init_streams(lcg, sd, 257)
        assert [int(v) for v in arr[[0, 1, 100, 256]]] == [orc.stream_start(lcg, sd, i) for i in (0, 1, 100, 256)]


# ------------------------------------------------------------ draw checksums

def test_checksum_equals_sum_of_skips(orc):
    """Sum of outputs X_1..X_n, recomputed through eq. (2) instead of iteration."""
    lcg = W.Lcg()
    counts = np.array([0, 1, 2, 7, 64, 300], dtype=np.uint32)
    for sd in (W.hash_seeding(), W.stride_seeding()):
        chk = orc.seed_and_draw(lcg, sd, counts)
        for i, n in enumerate(counts):
            x0 = orc.stream_start(lcg, sd, i)
            assert int(chk[i]) == sum(orc.skip(x0, d, G, 1, 63) for d in range(1, int(n) + 1)) & MASK64
    st = orc.init_streams(lcg, W.hash_seeding(), counts.size)
    start = st.copy()
    chk2 = orc.seed_and_draw(lcg, None, counts, states=st)
    assert np.array_equal(chk2, orc.seed_and_draw(lcg, W.hash_seeding(), counts))
    for i, n in enumerate(counts):
        assert int(st[i]) == orc.skip(int(start[i]), int(n), G, 1, 63)


def test_checksum_threads_independent(orc):
    lcg = W.Lcg()
    counts = W.draw_counts(4096, seed=42)
    a = orc.seed_and_draw(lcg, W.stride_seeding(), counts, threads=1)
    b = orc.seed_and_draw(lcg, W.stride_seeding(), counts, threads=7)
    assert np.array_equal(a, b)


# ------------------------------------------------------------ uniform and log

def test_uniform_mapping(orc):
    assert orc.uniform(0) == 2.0 ** -53
    assert orc.uniform(MASK63) == 1.0
    assert orc.uniform(1 << 62) == 0.5 + 2.0 ** -53
    rnd = random.Random(23)
    for _ in range(1000):
        x = rnd.getrandbits(63)
        assert orc.uniform(x) * 2.0 ** 53 == (x >> 10) + 1


def test_uniforms_brute_force(orc):
    """Row j of the uniforms is every stream's (j+1)-th output mapped to
    (0, 1]: recomputed with Python integers from each stream's start state
    (the LCG step written out as g x + 1 mod 2^63, the mapping as
    ((x >> 10) + 1) 2^-53), for both seedings and the load mode."""
    lcg = W.Lcg()
    n, k = 37, 9
    for sd in (W.hash_seeding(first_index=5), W.stride_seeding(first_index=11)):
        u = orc.uniforms(lcg, sd, n, k)
        assert u.shape == (k, n)
        for i in range(n):
            x = orc.stream_start(lcg, sd, i)
            for j in range(k):
                x = (G * x + 1) & MASK63
                assert u[j, i] == ((x >> 10) + 1) * 2.0 ** -53
    st = np.array([orc.stream_start(lcg, W.hash_seeding(), i) for i in range(n)], np.uint64)
    st0 = st.copy()
    u = orc.uniforms(lcg, None, n, k, st)
    assert np.array_equal(u, orc.uniforms(lcg, W.hash_seeding(), n, k))
    for i in range(n):
        x = int(st0[i])
        for _ in range(k):
            x = (G * x + 1) & MASK63
        assert int(st[i]) == x


def test_uniforms_moments(orc):
    """(0, 1], mean 1/2 and variance 1/12 within 5 standard errors over
    2^16 x 8 values."""
    u = orc.uniforms(W.Lcg(), W.hash_seeding(), 1 << 16, 8).ravel()
    assert u.min() > 0.0 and u.max() <= 1.0
    n = u.size
    assert abs(u.mean() - 0.5) < 5 * math.sqrt(1 / 12 / n)
    assert abs(u.var() - 1 / 12) < 5 * math.sqrt(1 / 180 / n)


def test_ln_accuracy_vs_mpmath(orc):
    mpmath.mp.prec = 160
    rng = np.random.default_rng(1)
    ks = [int(v) for v in rng.integers(1, 1 << 53, 4000)]
    ks += [1, 2, 3, (1 << 52) - 1, 1 << 52, (1 << 52) + 1, 3 << 50, (3 << 50) - 1, (3 << 50) + 1,
           3 << 51, (3 << 51) - 1, (1 << 53) - 1, (1 << 53) - 2]
    worst = 0.0
    for k in ks:
        u = k * 2.0 ** -53
        got = orc.ln(u)
        if u == 1.0:
            assert got == 0.0
            continue
        ex = mpmath.log(mpmath.mpf(u))
        err = float(abs(mpmath.mpf(got) - ex)) / float(np.spacing(abs(float(ex))))
        worst = max(worst, err)
    assert worst <= 1.25
    assert orc.ln(1.0) == 0.0
    for k in range(1, 54):
        assert abs(orc.ln(2.0 ** -k) - (-k * 0.6931471805599453)) <= 2 * np.spacing(k * 0.6931471805599453)


def test_u128_to_double_rounding(orc):
    cases = [0, 1, (1 << 53) - 1, 1 << 53, (1 << 53) + 1, (1 << 53) + 3, (1 << 54) + 2, (1 << 54) + 6,
             (1 << 64) - 1, 1 << 64, (1 << 100) + (1 << 47), (1 << 100) + (1 << 47) + 1,
             (1 << 128) - 1, 3 << 90]
    rnd = random.Random(29)
    cases += [rnd.getrandbits(rnd.randrange(1, 128)) for _ in range(3000)]
    for v in cases:
        assert orc.u128_to_f64(v) == float(v), v
