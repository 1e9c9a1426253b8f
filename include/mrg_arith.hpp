// MRG32k3a arithmetic shared by the kernels and the host side of the library.
//
// Generator (sec. 4.1; constants of L'Ecuyer 1999, which that section cites):
//   x1[n] = (a12 * x1[n-2] - a13n * x1[n-3]) mod m1
//   x2[n] = (a21 * x2[n-1] - a23n * x2[n-3]) mod m2
//   z[n]  = (x1[n] - x2[n]) mod m1, reported as m1 when 0
//
// gfx950 formulation.  Neither modulus is reduced with a division.  Both are
// pseudo-Mersenne: 2^32 = C (mod m) with C = 209 for m1 and 22853 for m2, so a
// 64-bit value hi*2^32 + lo folds to hi*C + lo.  Inside the hot loop a state
// word is any representative in [0, 2^32) of its residue ("lazy" form), which
// removes every conditional subtraction from the recurrence:
//   -x = ~x + 1 - 2^32 = ~x + (1 - C)  (mod m)  for every 32-bit x,
// so a*(-x) = a*~x + K with the constant K = a*(1 - C) mod m, and each
// product-sum is two v_mad_u64_u32 starting from K.  Folding then brings the
// 53-bit sum back to 32 bits (two folds for m1, three for m2).  Only the
// output combination and the state write-back map a word to its canonical
// residue, with min(x, x + C) (x + C wraps below x exactly when x >= m).
//
// A second formulation keeps the state in binary64 (the "F" functions):
// words are integer-valued doubles in [-5, m), every product-sum of them is
// below 2^53 in magnitude, so one FMA forms it exactly, and
// r = p - m * floor(p / m + bias) is exact (the biased quotient is the true
// one or one more) and lands back in [-5, m).  Each step is then five
// binary64 operations per component and five more for the combination.  Both
// formulations give the same residues.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define MRG_HD __host__ __device__ __forceinline__
#else
#define MRG_HD static inline
#endif

namespace mrg {

constexpr uint32_t M1 = 4294967087u;  // 2^32 - 209
constexpr uint32_t M2 = 4294944443u;  // 2^32 - 22853
constexpr uint32_t C1 = 209u;         // 2^32 mod m1
constexpr uint32_t C2 = 22853u;       // 2^32 mod m2
constexpr uint32_t A12 = 1403580u;
constexpr uint32_t A13N = 810728u;
constexpr uint32_t A21 = 527612u;
constexpr uint32_t A23N = 1370589u;
// K = a * (1 - C) mod m, the constant term of a*(-x) written as a*~x + K.
constexpr uint32_t K1 = (uint32_t)(((uint64_t)A13N * (uint64_t)(M1 - (C1 - 1u))) % M1);
constexpr uint32_t K2 = (uint32_t)(((uint64_t)A23N * (uint64_t)(M2 - (C2 - 1u))) % M2);
constexpr double NORM = 2.328306549295727688e-10;  // nearest double to 1/(m1+1)

MRG_HD uint32_t umin(uint32_t a, uint32_t b) { return a < b ? a : b; }

// Canonical residue of a lazy word: x mod m for x in [0, 2^32).
MRG_HD uint32_t canon1(uint32_t x) { return umin(x, x + C1); }
MRG_HD uint32_t canon2(uint32_t x) { return umin(x, x + C2); }

// Next component-1 word from x1[n-3] = s0 and x1[n-2] = s1 (both lazy);
// result lazy.  t < (a13n + a12 + 1) * 2^32 < 2^53.1; u < 2^32 + 2^29.
// The multipliers are parameters so that a kernel can pass copies held in
// vector registers.
MRG_HD uint32_t next1(uint32_t s0, uint32_t s1, uint32_t a13n = A13N, uint32_t a12 = A12)
{
    uint64_t t = (uint64_t)a13n * (uint32_t)~s0 + K1;
    t += (uint64_t)a12 * s1;
    uint64_t u = (uint64_t)(uint32_t)(t >> 32) * C1 + (uint32_t)t;
    return (uint32_t)u + (uint32_t)(u >> 32) * C1;
}

// Next component-2 word from x2[n-3] = s3 and x2[n-1] = s5 (both lazy);
// result lazy.  t < 2^52.9; u < 2^35.5; v < 2^32 + 2^18.1.
MRG_HD uint32_t next2(uint32_t s3, uint32_t s5, uint32_t a23n = A23N, uint32_t a21 = A21)
{
    uint64_t t = (uint64_t)a23n * (uint32_t)~s3 + K2;
    t += (uint64_t)a21 * s5;
    uint64_t u = (uint64_t)(uint32_t)(t >> 32) * C2 + (uint32_t)t;
    uint64_t v = (uint64_t)(uint32_t)(u >> 32) * C2 + (uint32_t)u;
    return (uint32_t)v + (uint32_t)(v >> 32) * C2;
}

// Combined output z' in [1, m1] from lazy x1[n], x2[n]:
// a = x1 mod m1, b = (x2 mod m2) + 1, y = a - b (mod 2^32);
// a >= b: z = y + 1;  a < b (x1 <= x2): z = y + 1 + m1 = y + 1 - 209 (mod 2^32).
MRG_HD uint32_t combine(uint32_t x1, uint32_t x2)
{
    uint32_t a = canon1(x1);
    uint32_t b = canon2(x2) + 1u;
    uint32_t y = a - b;
    return y + (a < b ? 1u - C1 : 1u);
}

MRG_HD double to_f64(uint32_t z) { return (double)z * NORM; }

// (2k + 1) * 2^-24 with k = (z - 1) >> 9 < 2^23: the binary32 number with
// exponent 0 and mantissa k is 1 + k * 2^-23, and subtracting 1 - 2^-24 from
// it is exact (the operands are within a factor of two, and the difference
// (2k + 1) * 2^-24 has at most 24 significant bits).
MRG_HD float to_f32(uint32_t z)
{
    const uint32_t k = (z - 1u) >> 9;
    return __builtin_bit_cast(float, 0x3F800000u | k) - 0x1.fffffep-1f;
}

// ---- matrix-vector product mod m for jumps (entries and x any 32-bit) ----
// p = M*x < 2^64 folds to hi*C + lo < 2^32 (C + 1); three of them sum below
// 2^48.2; one more fold leaves < 2^32 + 2^30.6, and the last fold is exact
// in 32 bits.  Result canonical.
template <uint32_t C>
MRG_HD uint32_t dot3_mod(uint32_t m0, uint32_t m1_, uint32_t m2_,
                         uint32_t x0, uint32_t x1, uint32_t x2)
{
    uint64_t p0 = (uint64_t)m0 * x0, p1 = (uint64_t)m1_ * x1, p2 = (uint64_t)m2_ * x2;
    uint64_t s = (uint64_t)(uint32_t)(p0 >> 32) * C + (uint32_t)p0;
    s += (uint64_t)(uint32_t)(p1 >> 32) * C + (uint32_t)p1;
    s += (uint64_t)(uint32_t)(p2 >> 32) * C + (uint32_t)p2;
    uint64_t u = (uint64_t)(uint32_t)(s >> 32) * C + (uint32_t)s;
    uint32_t r = (uint32_t)u + (uint32_t)(u >> 32) * C;
    return umin(r, r + C);
}

// v <- M v (mod m) for one component; M row-major 3x3.
template <uint32_t C>
MRG_HD void matvec3(const uint32_t *M, uint32_t &v0, uint32_t &v1, uint32_t &v2)
{
    uint32_t r0 = dot3_mod<C>(M[0], M[1], M[2], v0, v1, v2);
    uint32_t r1 = dot3_mod<C>(M[3], M[4], M[5], v0, v1, v2);
    uint32_t r2 = dot3_mod<C>(M[6], M[7], M[8], v0, v1, v2);
    v0 = r0; v1 = r1; v2 = r2;
}

// ---- binary64 formulation -------------------------------------------------
constexpr double M1D = 4294967087.0;
constexpr double M2D = 4294944443.0;
constexpr double INV1 = 1.0 / 4294967087.0;  // rounds above 1/m1: m1 * INV1 -> 1.0
constexpr double INV2 = 1.0 / 4294944443.0;

// The words are near-canonical: integer-valued doubles in [-5, m), each
// congruent to its residue.  A product-sum of such words stays below 2^53 in
// magnitude (at most 6.03e15 for component 1, 5.89e15 for component 2), so one
// FMA forms it exactly.  The quotient t = RN(p * INV + 2^-30) exceeds p/m by
// between 6.2e-10 and 1.25e-9 (|p/m| < 1.41e6 bounds both roundings by
// 3.2e-10), so floor(t) is the true quotient, or one more when the residue is
// within 5.4 of m; r = p - m * floor(t) is then exact and lies in [-5, m).
constexpr double QBIAS = 0x1p-30;

// Next component-1 word from x1[n-3] = s0 and x1[n-2] = s1.
MRG_HD double next1f(double s0, double s1)
{
    const double p = __builtin_fma((double)A12, s1, -((double)A13N * s0));
    return __builtin_fma(-__builtin_floor(__builtin_fma(p, INV1, QBIAS)), M1D, p);
}

// Next component-2 word from x2[n-3] = s3 and x2[n-1] = s5.
MRG_HD double next2f(double s3, double s5)
{
    const double p = __builtin_fma((double)A21, s5, -((double)A23N * s3));
    return __builtin_fma(-__builtin_floor(__builtin_fma(p, INV2, QBIAS)), M2D, p);
}

// Combined output z' in [1, m1] (as an exact binary64 integer) from
// near-canonical r1, r2.  x2 = r2 + m2 * [r2 < 0] is the canonical residue of
// r2 ([r2 < 0] = clamp(-r2, 0, 1), r2 being an integer); w = r1 - x2 lies in
// [-m2 - 4, m1 - 1] and is congruent to the combination mod m1, so
// z = w + m1 * [w <= 0] with [w <= 0] = clamp(1 - w, 0, 1) lands in
// [m1 - m2 - 4, m1], and w = 0 (equal residues) gives m1.
MRG_HD double combinef(double r1, double r2)
{
    const double c = __builtin_fmin(__builtin_fmax(-r2, 0.0), 1.0);
    const double w = r1 - __builtin_fma(c, M2D, r2);
    const double k = __builtin_fmin(__builtin_fmax(1.0 - w, 0.0), 1.0);
    return __builtin_fma(k, M1D, w);
}

// The same combination when r2 >= 0 (then r2 is already the canonical x2):
// w = r1 - r2 lies in [-m2 - 4, m1 - 1] (r1 >= -5 and r2 < m2) and is
// congruent to the combination mod m1, so z = w + m1 * [w <= 0] lands in
// [m1 - m2 - 4, m1] as above; three operations instead of five.  For
// r2 in [-5, 0) the result is wrong (x2 is r2 + m2 there); a caller that
// uses this form must detect that case (the sign bit of r2) and recompute
// with combinef.  The reductions give r2 < 0 only when the residue lies
// within about 5.4 of m2, about 5 times in 2^32 outputs.
MRG_HD double combinef_nn(double r1, double r2)
{
    const double w = r1 - r2;
    const double k = __builtin_fmin(__builtin_fmax(1.0 - w, 0.0), 1.0);
    return __builtin_fma(k, M1D, w);
}

// High word of a binary64 value: its sign bit is set for negative values
// (and for -0.0, which the reductions never produce: a false alarm at worst).
MRG_HD uint32_t hi_word(double x)
{
    return (uint32_t)(__builtin_bit_cast(uint64_t, x) >> 32);
}

// Canonical residue (as uint32) of a near-canonical word.
MRG_HD uint32_t canonf(double r, double m)
{
    const double c = __builtin_fmin(__builtin_fmax(-r, 0.0), 1.0);
    return (uint32_t)__builtin_fma(c, m, r);
}

MRG_HD double to_f64f(double z) { return z * NORM; }

// FP32 output from an exact binary64 z in [1, m1]: k = (z - 1) >> 9 taken as
// the truncated conversion of (z - 1) * 2^-9 (exact: at most 32 significant
// bits), then as to_f32.  The same value as to_f32((uint32_t)z), one
// instruction fewer.
MRG_HD float to_f32f(double z)
{
    const uint32_t k = (uint32_t)__builtin_fma(z, 0x1p-9, -0x1p-9);
    return __builtin_bit_cast(float, 0x3F800000u | k) - 0x1.fffffep-1f;
}

// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): the state advances by a fixed
// odd gamma and each output is a bijective mix of the new state, so output k
// of a generator seeded with s is mix(s + (k+1) * gamma).
// ---------------------------------------------------------------------------
constexpr uint64_t kSplitMixGamma = 0x9e3779b97f4a7c15ull;

MRG_HD uint64_t splitmix64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

MRG_HD uint64_t splitmix64_next(uint64_t &x)
{
    x += kSplitMixGamma;
    return splitmix64_mix(x);
}

// A 64-bit seed expanded into a valid state (random spacing, sec. 2.3):
// successive SplitMix64 outputs mod m1 for words 0-2 and mod m2 for words
// 3-5; a triple that comes out all zero (probability below 2^-95) is drawn
// again, as often as it takes (the generator's outputs are a bijection of
// its 2^64 states, so a nonzero triple always comes).
MRG_HD void expand_seed(uint64_t seed, uint32_t out[6])
{
    uint64_t x = seed;
    for (int c = 0; c < 2; ++c) {
        const uint64_t m = c ? M2 : M1;
        do {
            for (int i = 0; i < 3; ++i) out[3 * c + i] = (uint32_t)(splitmix64_next(x) % m);
        } while ((out[3 * c] | out[3 * c + 1] | out[3 * c + 2]) == 0u);
    }
}

}  // namespace mrg
