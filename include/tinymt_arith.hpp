// TinyMT32 arithmetic of the library: the generator, its published seeding,
// and the GF(2) polynomial arithmetic that checks parameter sets and places
// sub-streams.  Shared by the HIP kernels, the public device header
// (tinymt_device.h) and host builds for CPU tests.
//
// Method (paper sec. 4.2).  TinyMT is the small Mersenne-Twister offspring
// of Saito & Matsumoto (2011): a 127-bit state (four 32-bit words, bit 31 of
// word 0 outside the state), a GF(2)-linear transition and a non-linear
// tempering of the output, with independent generators obtained by
// parameterisation (mat1, mat2, tmat).  The paper's hybrid gives all threads
// of a group the same parameter set and hands each thread its own sub-stream
// of that generator by sequence splitting (sec. 2.3): the sequence is cut
// into equal chunks whose first states go to the threads by their index.
//
// Parameter sets.  Dynamic Creator's files are not at hand, so sets come from
// a search of our own: a candidate is accepted when the characteristic
// polynomial of its transition has degree 127 and is irreducible.  127 is a
// Mersenne exponent (2^127 - 1 is prime), so such a polynomial is primitive
// and every nonzero state has the full period 2^127 - 1.  The polynomial is
// found by the Berlekamp-Massey algorithm on a linear output bit of the
// state (254 terms, twice the degree), and irreducibility by Rabin's test for
// a prime degree n: x^(2^n) = x (mod phi) and phi has no root in GF(2).
//
// Jumps.  With phi the characteristic polynomial and T the transition,
// T^e s = T g(T) s for g(x) = x^(e-1) mod phi and any e >= 1: the extra
// transition clears the one bit (bit 31 of word 0) that the 127-dimensional
// arithmetic leaves undetermined.  g is r * prod_{i in bits(e)} x^(2^i) with
// r = x^-1 mod phi = (phi - 1) / x (phi(0) = 1), the powers x^(2^i) mod phi
// coming from the parameter set's table, and g(T) s is evaluated by Horner's
// rule (a transition per coefficient).
//
// Polynomials are 128-bit values in four words: bit b of word k is the
// coefficient of x^(32k + b).  Residues mod phi have degree below 127.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define TMT_HD __host__ __device__ __forceinline__
#else
#define TMT_HD static inline
#endif

namespace mrg {
namespace tmt {

constexpr uint32_t kMask = 0x7fffffffu;  // the state bits of word 0
constexpr int kJumpBits = 192;           // exponents below 2^192

// A parameter set's device record (kRecordWords words):
//   [0..3]   mat1, mat2, tmat, 0
//   [4..7]   phi, the characteristic polynomial (degree 127: bit 127 set)
//   [8 + 4i .. 8 + 4i + 3]   x^(2^i) mod phi, i in [0, kJumpBits)
constexpr int kRecordWords = 8 + 4 * kJumpBits;
constexpr int kRecPhi = 4;
constexpr int kRecPow = 8;

// ---------------------------------------------------------------------------
// The generator
// ---------------------------------------------------------------------------
// One transition: x = (s0 & mask) ^ s1 ^ s2, x ^= x << 1,
// y = s3 ^ (s3 >> 1) ^ x; the words move down one place, the new s2 is
// x ^ (y << 10), the new s3 is y, and when y is odd mat1 and mat2 are added
// to the new s1 and s2.
TMT_HD void step(uint32_t &s0, uint32_t &s1, uint32_t &s2, uint32_t &s3, uint32_t mat1,
                 uint32_t mat2)
{
    uint32_t x = (s0 & kMask) ^ s1 ^ s2;
    x ^= x << 1;
    const uint32_t y = s3 ^ (s3 >> 1) ^ x;
    const uint32_t odd = 0u - (y & 1u);
    s0 = s1;
    s1 = s2 ^ (odd & mat1);
    s2 = x ^ (y << 10) ^ (odd & mat2);
    s3 = y;
}

TMT_HD void step(uint32_t s[4], uint32_t mat1, uint32_t mat2)
{
    step(s[0], s[1], s[2], s[3], mat1, mat2);
}

// Output word of a state: t = s0 + (s2 >> 8) (an integer addition, the
// non-linear part), s3 ^ t, and tmat added when t is odd.
TMT_HD uint32_t temper(uint32_t s0, uint32_t s2, uint32_t s3, uint32_t tmat)
{
    const uint32_t t = s0 + (s2 >> 8);
    return s3 ^ t ^ ((0u - (t & 1u)) & tmat);
}

// FP32 (2 * (w >> 9) + 1) * 2^-24 and FP64 (2w + 1) * 2^-33: exact, in (0, 1).
TMT_HD float to_f32(uint32_t w)
{
    return (float)(2u * (w >> 9) + 1u) * 0x1p-24f;
}
TMT_HD double to_f64(uint32_t w)
{
    return ((double)w * 2.0 + 1.0) * 0x1p-33;
}

// Published seeding of a status from a 32-bit seed: words (seed, mat1, mat2,
// tmat), seven rounds of s[i % 4] ^= i + 1812433253 * (p ^ (p >> 30)) with p
// the word before, an all-zero state replaced by the letters T, I, N, Y, then
// eight transitions.
TMT_HD void seed_status(uint32_t seed, uint32_t mat1, uint32_t mat2, uint32_t tmat,
                        uint32_t s[4])
{
    s[0] = seed;
    s[1] = mat1;
    s[2] = mat2;
    s[3] = tmat;
    for (uint32_t i = 1; i < 8; ++i) {
        const uint32_t p = s[(i - 1) & 3u];
        s[i & 3u] ^= i + 1812433253u * (p ^ (p >> 30));
    }
    if (((s[0] & kMask) | s[1] | s[2] | s[3]) == 0u) {
        s[0] = 0x54u;
        s[1] = 0x49u;
        s[2] = 0x4Eu;
        s[3] = 0x59u;
    }
    for (int i = 0; i < 8; ++i) step(s, mat1, mat2);
}

// SplitMix64 output k of a generator seeded with `seed` (Steele, Lea & Flood,
// OOPSLA 2014): the finaliser applied to seed + (k + 1) * gamma.
TMT_HD uint64_t splitmix_at(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1u) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Candidate c of the parameter search under master seed m: SplitMix64
// outputs 2c and 2c+1 of seed m + 1; mat1 and mat2 are the low and high
// halves of the first, tmat the low half of the second.
TMT_HD void candidate(uint64_t master, uint64_t c, uint32_t p[3])
{
    const uint64_t a = splitmix_at(master + 1u, 2u * c);
    const uint64_t b = splitmix_at(master + 1u, 2u * c + 1u);
    p[0] = (uint32_t)a;
    p[1] = (uint32_t)(a >> 32);
    p[2] = (uint32_t)b;
}

// The 32-bit seed of parameter set q's base status: the low half of
// SplitMix64 output q of the master seed.
TMT_HD uint32_t set_seed(uint64_t master, uint64_t q)
{
    return (uint32_t)splitmix_at(master, q);
}

// ---------------------------------------------------------------------------
// Polynomials over GF(2)
// ---------------------------------------------------------------------------
// a <- a * x mod phi for a residue a (degree < 127): shift up one place and
// add phi when the coefficient of x^127 came out set.
TMT_HD void mulx(uint32_t a[4], const uint32_t phi[4])
{
    const uint32_t top = 0u - ((a[3] >> 30) & 1u);
    a[3] = ((a[3] << 1) | (a[2] >> 31)) ^ (phi[3] & top);
    a[2] = ((a[2] << 1) | (a[1] >> 31)) ^ (phi[2] & top);
    a[1] = ((a[1] << 1) | (a[0] >> 31)) ^ (phi[1] & top);
    a[0] = (a[0] << 1) ^ (phi[0] & top);
}

// r = a * b mod phi (residues a, b): Horner's rule over the coefficients of
// a from the top down, r <- r * x + a_i * b (the coefficient of x^127 of a
// residue is 0, so starting there adds nothing).  Words are indexed by
// constants only, so that device code keeps the operands in registers.
TMT_HD void mulmod(const uint32_t a[4], const uint32_t b[4], const uint32_t phi[4],
                   uint32_t r[4])
{
    const uint32_t b0 = b[0], b1 = b[1], b2 = b[2], b3 = b[3];
    uint32_t t[4] = {0u, 0u, 0u, 0u};
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
#endif
    for (int w = 3; w >= 0; --w) {
        const uint32_t aw = a[w];
        for (int i = 31; i >= 0; --i) {
            mulx(t, phi);
            const uint32_t take = 0u - ((aw >> i) & 1u);
            t[0] ^= b0 & take;
            t[1] ^= b1 & take;
            t[2] ^= b2 & take;
            t[3] ^= b3 & take;
        }
    }
    r[0] = t[0]; r[1] = t[1]; r[2] = t[2]; r[3] = t[3];
}

TMT_HD uint32_t rev32(uint32_t v)
{
    v = ((v >> 1) & 0x55555555u) | ((v & 0x55555555u) << 1);
    v = ((v >> 2) & 0x33333333u) | ((v & 0x33333333u) << 2);
    v = ((v >> 4) & 0x0F0F0F0Fu) | ((v & 0x0F0F0F0Fu) << 4);
    v = ((v >> 8) & 0x00FF00FFu) | ((v & 0x00FF00FFu) << 8);
    return (v >> 16) | (v << 16);
}

// Characteristic polynomial of the transition of parameters p, from the
// Berlekamp-Massey algorithm on bit 0 of s3 over 254 transitions from a fixed
// nonzero state.  Returns the linear complexity L (127 for every set worth
// keeping) and, when L = 127, phi(x) = x^127 C(1/x) for the connection
// polynomial C found (phi = 0 otherwise).  Bit vectors of 256 bits (8 words); the shifted copy
// Bs = x^m B of the last connection polynomial moves up one place per step.
TMT_HD int charpoly(const uint32_t p[3], uint32_t phi[4])
{
    uint32_t s[4] = {0x12345678u, 0x9abcdef0u, 0x0fedcba9u, 0x87654321u};
    uint32_t C[8] = {1u, 0, 0, 0, 0, 0, 0, 0};
    uint32_t Bs[8] = {2u, 0, 0, 0, 0, 0, 0, 0};
    uint32_t H[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // bit i: the term i steps back
    int L = 0;
    for (int k = 0; k < 254; ++k) {
        step(s, p[0], p[1]);
        const uint32_t a = s[3] & 1u;
        for (int w = 7; w > 0; --w) H[w] = (H[w] << 1) | (H[w - 1] >> 31);
        H[0] = (H[0] << 1) | a;
        uint32_t par = 0;  // discrepancy: parity of sum_i C_i a_(k-i)
        for (int w = 0; w < 8; ++w) par ^= C[w] & H[w];
        par ^= par >> 16;
        par ^= par >> 8;
        par ^= par >> 4;
        par ^= par >> 2;
        par ^= par >> 1;
        const bool d = (par & 1u) != 0u;
        if (d && 2 * L <= k) {
            uint32_t T[8];
            for (int w = 0; w < 8; ++w) {
                T[w] = C[w];
                C[w] ^= Bs[w];
            }
            L = k + 1 - L;
            Bs[0] = T[0] << 1;
            for (int w = 1; w < 8; ++w) Bs[w] = (T[w] << 1) | (T[w - 1] >> 31);
        } else {
            if (d)
                for (int w = 0; w < 8; ++w) C[w] ^= Bs[w];
            for (int w = 7; w > 0; --w) Bs[w] = (Bs[w] << 1) | (Bs[w - 1] >> 31);
            Bs[0] <<= 1;
        }
    }
    // L = 127: phi(x) = x^127 C(1/x), the 128 coefficients of C reversed
    const bool full = L == 127;
    phi[0] = full ? rev32(C[3]) : 0u;
    phi[1] = full ? rev32(C[2]) : 0u;
    phi[2] = full ? rev32(C[1]) : 0u;
    phi[3] = full ? rev32(C[0]) : 0u;
    return L;
}

// phi of degree 127 is irreducible (Rabin, prime degree): phi(0) = 1, an odd
// number of terms (phi(1) = 1) and x^(2^127) = x mod phi.
TMT_HD bool irreducible127(const uint32_t phi[4])
{
    if (!(phi[3] >> 31) || !(phi[0] & 1u)) return false;
    uint32_t ones = 0;
    for (int w = 0; w < 4; ++w) {
        uint32_t v = phi[w];
        v ^= v >> 16;
        v ^= v >> 8;
        v ^= v >> 4;
        v ^= v >> 2;
        v ^= v >> 1;
        ones ^= v & 1u;
    }
    if (!ones) return false;
    uint32_t t[4] = {2u, 0u, 0u, 0u};  // x
    for (int i = 0; i < 127; ++i) {
        uint32_t u[4];
        mulmod(t, t, phi, u);
        t[0] = u[0]; t[1] = u[1]; t[2] = u[2]; t[3] = u[3];
    }
    return t[0] == 2u && t[1] == 0u && t[2] == 0u && t[3] == 0u;
}

// A parameter set is kept when its characteristic polynomial has degree 127
// and is irreducible (period 2^127 - 1).
TMT_HD bool params_ok(const uint32_t p[3], uint32_t phi[4])
{
    return charpoly(p, phi) == 127 && irreducible127(phi);
}

// ---------------------------------------------------------------------------
// Jumps
// ---------------------------------------------------------------------------
// s <- T^e s for e = e0 + e1 * 2^64 + e2 * 2^128 (any e below 2^192), with
// p the set's parameters, phi its characteristic polynomial and pow its table
// of x^(2^i) mod phi (4 words each, i in [0, 192)).
TMT_HD void jump(uint32_t s[4], uint32_t mat1, uint32_t mat2, const uint32_t phi[4],
                 const uint32_t *pow, uint64_t e0, uint64_t e1, uint64_t e2)
{
    if ((e0 | e1 | e2) == 0u) return;
    // g = x^-1 * prod x^(2^i) over the bits of e
    uint32_t g[4] = {(phi[0] >> 1) | (phi[1] << 31), (phi[1] >> 1) | (phi[2] << 31),
                     (phi[2] >> 1) | (phi[3] << 31), phi[3] >> 1};
    const uint64_t ew[3] = {e0, e1, e2};
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
#endif
    for (int w = 0; w < 3; ++w) {
        uint64_t bits = ew[w];
        while (bits) {
            const int i = 64 * w + (int)__builtin_ctzll(bits);
            bits &= bits - 1u;
            uint32_t u[4];
            mulmod(g, pow + 4 * i, phi, u);
            g[0] = u[0]; g[1] = u[1]; g[2] = u[2]; g[3] = u[3];
        }
    }
    // Horner: acc = g(T) s, then one more transition
    const uint32_t x0 = s[0], x1 = s[1], x2 = s[2], x3 = s[3];
    uint32_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
#endif
    for (int w = 3; w >= 0; --w) {
        const uint32_t gw = g[w];
        for (int i = 31; i >= 0; --i) {
            step(a0, a1, a2, a3, mat1, mat2);
            const uint32_t take = 0u - ((gw >> i) & 1u);
            a0 ^= x0 & take;
            a1 ^= x1 & take;
            a2 ^= x2 & take;
            a3 ^= x3 & take;
        }
    }
    step(a0, a1, a2, a3, mat1, mat2);
    s[0] = a0; s[1] = a1; s[2] = a2; s[3] = a3;
}

// The table of a record: pow[i] = x^(2^i) mod phi, by repeated squaring.
TMT_HD void pow_table(const uint32_t phi[4], uint32_t *pow)
{
    uint32_t t[4] = {2u, 0u, 0u, 0u};
    for (int i = 0; i < kJumpBits; ++i) {
        pow[4 * i + 0] = t[0];
        pow[4 * i + 1] = t[1];
        pow[4 * i + 2] = t[2];
        pow[4 * i + 3] = t[3];
        uint32_t u[4];
        mulmod(t, t, phi, u);
        t[0] = u[0]; t[1] = u[1]; t[2] = u[2]; t[3] = u[3];
    }
}

}  // namespace tmt
}  // namespace mrg
