// Device-side random-number primitives for gfx950.
//
// Method: Cuneo & Variansyah, "An Alternative to Stride-Based RNG for Monte
// Carlo Transport" (arXiv 2403.06362).
//   lcg_next ....... eq. (1), X <- (g X + c) mod 2^m; the new state is the output
//   affine_apply ... one factor of the skip-ahead of eq. (2): X <- G X + C mod 2^m
//   murmur_hash .... Listing 1, hash(k, s) with wrapping 64-bit multiplies
//   to_uniform ..... top 53 state bits, plus one, times 2^-53 (exact, in (0, 1])
//   fixed_log ...... natural log with a fixed IEEE operation sequence
//
// All 64-bit products are the low 64 bits of the full product; reduction
// modulo 2^m is a mask because 2^m divides 2^64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcrng {

struct LcgDev {
    uint64_t g;
    uint64_t c;
    uint64_t mask;      // 2^m - 1 (all ones for m = 64)
    uint32_t shift53;   // m - 53: right shift that keeps the top 53 state bits
    uint32_t m;
};

__device__ __forceinline__ uint64_t lcg_next(const LcgDev& L, uint64_t x) {
    return (L.g * x + L.c) & L.mask;
}

// The same step for m >= 32, where the mask leaves the low word alone (one
// AND on the high word instead of two).
__device__ __forceinline__ uint64_t lcg_next_wide(const LcgDev& L, uint64_t x) {
    return (L.g * x + L.c) & (L.mask | 0xffffffffull);
}

__device__ __forceinline__ uint64_t affine_apply(uint64_t G, uint64_t C, uint64_t mask, uint64_t x) {
    return (G * x + C) & mask;
}

constexpr uint64_t kMurmurM = 0xC6A4A7935BD1E995ull;

__host__ __device__ __forceinline__ uint64_t murmur_sub(uint64_t x) {
    const uint64_t y = x * kMurmurM;
    return y ^ (y >> 47);
}

// seed_hash = subhash(s ^ 8M) depends on the seed only; callers hoist it.
__host__ __device__ __forceinline__ uint64_t murmur_seed_part(uint64_t s) {
    return murmur_sub(s ^ (8ull * kMurmurM));
}

// The steps of hash(k, s) after the first product y = k M.
__host__ __device__ __forceinline__ uint64_t murmur_from_product(uint64_t y, uint64_t seed_part) {
    return murmur_sub(seed_part ^ ((y ^ (y >> 47)) * kMurmurM));
}

__host__ __device__ __forceinline__ uint64_t murmur_with_seed_part(uint64_t k, uint64_t seed_part) {
    return murmur_from_product(k * kMurmurM, seed_part);
}

__host__ __device__ __forceinline__ uint64_t murmur_hash(uint64_t k, uint64_t s) {
    return murmur_with_seed_part(k, murmur_seed_part(s));
}

// u = ((X >> (m - 53)) + 1) * 2^-53.  The integer is at most 2^53, so the
// conversion to double is exact.
// The integer's halves are converted separately and joined by one fused
// multiply-add, hi 2^32 + lo, exact (as the plain conversion is) below 2^53.
__device__ __forceinline__ double to_uniform(const LcgDev& L, uint64_t x) {
    const uint64_t top = (x >> L.shift53) + 1ull;
    const double hi = static_cast<double>(static_cast<uint32_t>(top >> 32));
    const double lo = static_cast<double>(static_cast<uint32_t>(top));
    return __builtin_fma(hi, 0x1p32, lo) * 0x1p-53;
}

// ------------------------------------------------------------ division
// A correctly rounded quotient a / b is, on this hardware, the reciprocal
// r = rcp(b) refined by Newton steps r <- r + r (1 - b r) (two in double
// precision, one in single), the product q = a r and residual corrections
// q <- q + (a - b q) r (one in double, two in single), each a fused
// multiply-add, wrapped in operand scaling that acts only near the ends of
// the exponent range.  The refined reciprocal depends on b alone, so a
// divisor used many times (a cell's sigma_t, a flight's direction cosine)
// has it computed once.  quot(a, b, recip_refined(b)) then equals a / b bit
// for bit wherever the scaling does not act, which holds when |a| is at
// least 2^-900 (single: 2^-60), b is nonzero with |b| in [2^-64, 2^64] and
// |a| is at most 2^42: what the transport's validated geometry allows.  A
// smaller |a| (zero included) takes the plain division.
__device__ __forceinline__ double recip_refined(double b) {
    double r = __builtin_amdgcn_rcp(b);
    r = __builtin_fma(r, __builtin_fma(-b, r, 1.0), r);
    r = __builtin_fma(r, __builtin_fma(-b, r, 1.0), r);
    return r;
}

__device__ __forceinline__ double quot(double a, double b, double r) {
    if (!(__builtin_fabs(a) >= 0x1p-900)) return a / b;
    const double q = a * r;
    return __builtin_fma(__builtin_fma(-b, q, a), r, q);
}

__device__ __forceinline__ float recip_refined(float b) {
    const float r = __builtin_amdgcn_rcpf(b);
    return __builtin_fmaf(__builtin_fmaf(-b, r, 1.0f), r, r);
}

__device__ __forceinline__ float quot(float a, float b, float r) {
    if (!(__builtin_fabsf(a) >= 0x1p-60f)) return a / b;
    float q = a * r;
    q = __builtin_fmaf(__builtin_fmaf(-b, q, a), r, q);
    return __builtin_fmaf(__builtin_fmaf(-b, q, a), r, q);
}

// Natural logarithm of u in (0, 1] (any positive normal double works).
// Fixed sequence of IEEE double operations, each rounded to nearest, no
// fused multiply-add (the library is compiled with -ffp-contract=off):
//   u = f 2^e, f in [1, 2); f >= 3/2 -> f/2, e+1;  a = f - 1 (exact)
//   s = a / (2 + a);  w = s s;  p = 2/23, then p = p w + 2/(2k+1) for
//   k = 10 .. 1 (multiply and add rounded separately);  h = w p;
//   ln(1 + a) = a - s (a - h);  ln u = e LN2_HI + (ln(1 + a) + e LN2_LO)
// ln(1 + a) = 2 atanh(s) = 2s + sum_k 2 s^(2k+1)/(2k+1) and 2s = a - a s.
// LN2_HI is ln 2 truncated to 40 fraction bits, LN2_LO the double nearest
// to the rest.  Within 1.25 ulp of the exact logarithm.
__device__ __forceinline__ double fixed_log(double u) {
    constexpr double kLn2Hi = 0x1.62e42fefa2000p-1;
    constexpr double kLn2Lo = 0x1.9ef35793c7673p-41;
    constexpr double kC[12] = {0.0,        2.0 / 3.0,  2.0 / 5.0,  2.0 / 7.0,
                               2.0 / 9.0,  2.0 / 11.0, 2.0 / 13.0, 2.0 / 15.0,
                               2.0 / 17.0, 2.0 / 19.0, 2.0 / 21.0, 2.0 / 23.0};
    const uint64_t bits = __double_as_longlong(u);
    int e = static_cast<int>((bits >> 52) & 0x7ff) - 1023;
    double f = __longlong_as_double(static_cast<long long>((bits & 0x000fffffffffffffull) |
                                                           0x3ff0000000000000ull));
    if (f >= 1.5) {
        f = f * 0.5;
        e = e + 1;
    }
    const double a = f - 1.0;
    const double b = 2.0 + a;
    const double s = quot(a, b, recip_refined(b));   // a in {0} or [2^-53, 1/2), b in [7/4, 5/2)
    const double w = s * s;
    double p = kC[11];
#pragma unroll
    for (int k = 10; k >= 1; --k) {
        p = p * w;
        p = p + kC[k];
    }
    const double h = w * p;
    const double t = a - h;
    const double c = s * t;
    const double l = a - c;
    const double ed = static_cast<double>(e);
    const double r = l + ed * kLn2Lo;
    return ed * kLn2Hi + r;
}

// Quantised track length: q = round-half-even(s * 2^56) for 0 <= s < 2^7.
__device__ __forceinline__ uint64_t quantise(double s) {
    return static_cast<uint64_t>(__builtin_rint(s * 0x1p56));
}

}  // namespace mcrng
