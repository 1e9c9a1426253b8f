/*
 * MRG32k3a CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is the plain, slow, single-threaded definition of what the GPU
 * library computes.  Only the tests, the smoke check and the benchmark's CPU
 * baseline may load it.  It shares no code, header, table or constant
 * generator with the GPU library: every step is written out from the
 * definition with plain 64-bit integer `%`, one value at a time.
 *
 * Method (Passerat-Palmbach & Hill, HPCS 2012):
 *  - sec. 4.1 "MRG32k3a": the generator keeps 6 integers of state, has a
 *    period of about 2^191, and is split into 2^64 adjacent streams of 2^127
 *    numbers, each divided into substreams of 2^76 numbers (sequence
 *    splitting, sec. 2.3).  The paper cites L'Ecuyer 1999 for the generator
 *    itself; the moduli and multipliers below are that publication's values
 *    (the paper does not print them).
 *  - sec. 2.3 "Partitioning techniques": sequence splitting needs a jump
 *    ahead, which for a linear recurrence mod m is a matrix power mod m;
 *    random spacing seeds the same generator from different random states.
 *  - sec. 5 / Listing 1: a thread's RNG object returns the next number of its
 *    own stream, converted to the requested type (float in the listing).
 *
 * Readings of points the paper leaves open (each one also documented in the
 * design notes):
 *  - state order is oldest first: (x1[n-3], x1[n-2], x1[n-1],
 *    x2[n-3], x2[n-2], x2[n-1]);
 *  - output number 0 is produced by the first step (the seed is never
 *    emitted);
 *  - the combined integer output z = (x1 - x2) mod m1 is replaced by m1 when
 *    it is 0, so the uint32 output lies in [1, m1];
 *  - FP64 output: (double)z * NORM, NORM the double nearest 1/(m1+1), one
 *    IEEE round-to-nearest multiply;
 *  - FP32 output: k = (z - 1) >> 9, value (2k + 1) * 2^-24 (exact);
 *  - a 64-bit master seed is expanded into the 6 state words with SplitMix64
 *    (Steele, Lea & Flood, OOPSLA 2014): successive outputs w taken mod m1
 *    for the first triple and mod m2 for the second; an all-zero triple is
 *    redrawn.
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fno-fast-math -shared -fPIC.
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>

/* L'Ecuyer 1999, as cited in sec. 4.1. */
#define ORC_M1   4294967087ULL   /* 2^32 - 209   */
#define ORC_M2   4294944443ULL   /* 2^32 - 22853 */
#define ORC_A12  1403580ULL      /* x1[n] uses  a12 * x1[n-2] */
#define ORC_A13N 810728ULL       /*        and -a13n * x1[n-3] */
#define ORC_A21  527612ULL       /* x2[n] uses  a21 * x2[n-1] */
#define ORC_A23N 1370589ULL      /*        and -a23n * x2[n-3] */
#define ORC_NORM 2.328306549295727688e-10   /* nearest double to 1/(m1+1) */

enum { ORC_U32 = 0, ORC_F32 = 1, ORC_F64 = 2 };
enum { ORC_STREAM_MAJOR = 0, ORC_INTERLEAVED = 1 };

static uint64_t orc_modulus(int comp) { return comp == 0 ? ORC_M1 : ORC_M2; }

/* ---------------------------------------------------------------------- */
/* One step of the recurrence (sec. 4.1; L'Ecuyer 1999).                   */
/* s[0..2] = x1[n-3..n-1] in [0,m1), s[3..5] = x2[n-3..n-1] in [0,m2).     */
/* Returns the combined integer output z' in [1, m1].                      */
/* ---------------------------------------------------------------------- */
uint32_t orc_step(uint32_t s[6])
{
    int64_t p1 = (int64_t)(ORC_A12 * s[1]) - (int64_t)(ORC_A13N * s[0]);
    p1 %= (int64_t)ORC_M1;
    if (p1 < 0) p1 += (int64_t)ORC_M1;

    int64_t p2 = (int64_t)(ORC_A21 * s[5]) - (int64_t)(ORC_A23N * s[3]);
    p2 %= (int64_t)ORC_M2;
    if (p2 < 0) p2 += (int64_t)ORC_M2;

    s[0] = s[1]; s[1] = s[2]; s[2] = (uint32_t)p1;
    s[3] = s[4]; s[4] = s[5]; s[5] = (uint32_t)p2;

    int64_t z = (p1 - p2) % (int64_t)ORC_M1;
    if (z < 0) z += (int64_t)ORC_M1;
    if (z == 0) z = (int64_t)ORC_M1;
    return (uint32_t)z;
}

/* Output conversions of one integer output z' in [1, m1]. */
double orc_to_f64(uint32_t z) { return (double)z * ORC_NORM; }

float orc_to_f32(uint32_t z)
{
    uint32_t k = (z - 1u) >> 9;                 /* 0 .. 2^23 - 1 */
    return (float)(2u * k + 1u) * 0x1p-24f;     /* exact: 24-bit odd integer */
}

/* ---------------------------------------------------------------------- */
/* Fill: n outputs from each of S streams (states row-major [S][6]).        */
/* stream-major: out[s*n + k]; interleaved: out[k*S + s].                   */
/* Each state is advanced by n.                                             */
/* ---------------------------------------------------------------------- */
void orc_fill(uint32_t *states, uint64_t S, uint64_t n, int dtype, int layout,
              void *out)
{
    for (uint64_t s = 0; s < S; ++s) {
        uint32_t *st = states + 6 * s;
        for (uint64_t k = 0; k < n; ++k) {
            uint32_t z = orc_step(st);
            uint64_t idx = (layout == ORC_STREAM_MAJOR) ? s * n + k : k * S + s;
            if (dtype == ORC_U32)      ((uint32_t *)out)[idx] = z;
            else if (dtype == ORC_F32) ((float *)out)[idx] = orc_to_f32(z);
            else                       ((double *)out)[idx] = orc_to_f64(z);
        }
    }
}

/* Sample of one stream: outputs k0 .. k0+cnt-1 starting from state st
 * (advanced by k0 by stepping, not by jumping).  Used for sampled checks. */
void orc_skip(uint32_t st[6], uint64_t k)
{
    for (uint64_t i = 0; i < k; ++i) (void)orc_step(st);
}

/* ---------------------------------------------------------------------- */
/* Jump ahead (sec. 2.3 sequence splitting; sec. 4.1 streams/substreams).  */
/* Each component is x[n] = A_c x[n-1] on the column vector                */
/* (x[n-3], x[n-2], x[n-1]); A_c is the companion matrix of the recurrence.*/
/* A_c^e mod m_c by square-and-multiply over the bits of a 192-bit e.      */
/* ---------------------------------------------------------------------- */
void orc_companion(int comp, uint32_t A[9])
{
    memset(A, 0, 9 * sizeof(uint32_t));
    A[0 * 3 + 1] = 1;
    A[1 * 3 + 2] = 1;
    if (comp == 0) {
        A[2 * 3 + 0] = (uint32_t)(ORC_M1 - ORC_A13N);
        A[2 * 3 + 1] = (uint32_t)ORC_A12;
        A[2 * 3 + 2] = 0;
    } else {
        A[2 * 3 + 0] = (uint32_t)(ORC_M2 - ORC_A23N);
        A[2 * 3 + 1] = 0;
        A[2 * 3 + 2] = (uint32_t)ORC_A21;
    }
}

static void orc_matmul(uint64_t m, const uint32_t X[9], const uint32_t Y[9],
                       uint32_t R[9])
{
    uint32_t T[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            uint64_t acc = 0;
            for (int k = 0; k < 3; ++k)
                acc += ((uint64_t)X[i * 3 + k] * (uint64_t)Y[k * 3 + j]) % m;
            T[i * 3 + j] = (uint32_t)(acc % m);
        }
    memcpy(R, T, sizeof T);
}

void orc_matpow(int comp, const uint64_t e[3], uint32_t R[9])
{
    uint64_t m = orc_modulus(comp);
    uint32_t B[9];
    orc_companion(comp, B);
    memset(R, 0, 9 * sizeof(uint32_t));
    R[0] = R[4] = R[8] = 1;
    for (int w = 0; w < 3; ++w)
        for (int b = 0; b < 64; ++b) {
            if ((e[w] >> b) & 1u) orc_matmul(m, R, B, R);
            orc_matmul(m, B, B, B);
        }
}

void orc_matvec(int comp, const uint32_t M[9], uint32_t v[3])
{
    uint64_t m = orc_modulus(comp);
    uint32_t r[3];
    for (int i = 0; i < 3; ++i) {
        uint64_t acc = 0;
        for (int k = 0; k < 3; ++k)
            acc += ((uint64_t)M[i * 3 + k] * (uint64_t)v[k]) % m;
        r[i] = (uint32_t)(acc % m);
    }
    memcpy(v, r, sizeof r);
}

/* state <- A^e state, e a 192-bit little-endian exponent (3 words). */
void orc_jump(uint32_t s[6], const uint64_t e[3])
{
    uint32_t M[9];
    orc_matpow(0, e, M);
    orc_matvec(0, M, s);
    orc_matpow(1, e, M);
    orc_matvec(1, M, s + 3);
}

/* Jump every one of S states (row-major [S][6]) by its own exponent
 * (e: [S][3] words) or, when e_stride == 0, by the one exponent e[0..2]. */
void orc_jump_many(uint32_t *states, uint64_t S, const uint64_t *e, int e_stride)
{
    for (uint64_t s = 0; s < S; ++s)
        orc_jump(states + 6 * s, e + (e_stride ? 3 * s : 0));
}

/* Every one of S states jumped by the one exponent e: A^e formed once, then
 * one matrix-vector product per state and component. */
void orc_jump_uniform(uint32_t *states, uint64_t S, const uint64_t e[3])
{
    uint32_t P1[9], P2[9];
    orc_matpow(0, e, P1);
    orc_matpow(1, e, P2);
    for (uint64_t s = 0; s < S; ++s) {
        orc_matvec(0, P1, states + 6 * s);
        orc_matvec(1, P2, states + 6 * s + 3);
    }
}

/* Start of stream g: A^(g * 2^127) applied to the base state (sec. 4.1).
 * g * 2^127 = (g >> 1) * 2^128 + (g & 1) * 2^127. */
void orc_stream_start(const uint32_t base[6], uint64_t g, uint32_t out[6])
{
    uint64_t e[3] = { 0, (g & 1u) << 63, g >> 1 };
    memcpy(out, base, 6 * sizeof(uint32_t));
    orc_jump(out, e);
}

/* States of streams first .. first+S-1 of the set rooted at base. */
void orc_streams(const uint32_t base[6], uint64_t first, uint64_t S,
                 uint32_t *out)
{
    for (uint64_t i = 0; i < S; ++i)
        orc_stream_start(base, first + i, out + 6 * i);
}

/* The same starts stepped one stream at a time: stream g+1 begins 2^127
 * outputs after stream g (adjacent streams, sec. 4.1), so after the first
 * start each is one product by A^(2^127) of the one before. */
void orc_streams_adjacent(const uint32_t base[6], uint64_t first, uint64_t S,
                          uint32_t *out)
{
    if (S == 0) return;
    orc_stream_start(base, first, out);
    const uint64_t e[3] = { 0, (uint64_t)1 << 63, 0 };
    uint32_t P1[9], P2[9];
    orc_matpow(0, e, P1);
    orc_matpow(1, e, P2);
    for (uint64_t i = 1; i < S; ++i) {
        memcpy(out + 6 * i, out + 6 * (i - 1), 6 * sizeof(uint32_t));
        orc_matvec(0, P1, out + 6 * i);
        orc_matvec(1, P2, out + 6 * i + 3);
    }
}

/* ---------------------------------------------------------------------- */
/* Random spacing from a 64-bit master seed (sec. 2.3), via SplitMix64     */
/* (Steele, Lea & Flood 2014): gamma 0x9e3779b97f4a7c15 added to the       */
/* state, then the 64-bit finaliser (shift 30, multiply, shift 27,         */
/* multiply, shift 31).                                                    */
/* ---------------------------------------------------------------------- */
uint64_t orc_splitmix64_next(uint64_t *x)
{
    uint64_t z = (*x += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

void orc_seed_from_master(uint64_t master, uint32_t out[6])
{
    uint64_t x = master;
    for (int c = 0; c < 2; ++c) {
        uint64_t m = orc_modulus(c);
        for (;;) {
            uint32_t t[3];
            for (int i = 0; i < 3; ++i)
                t[i] = (uint32_t)(orc_splitmix64_next(&x) % m);
            if (t[0] | t[1] | t[2]) {
                memcpy(out + 3 * c, t, sizeof t);
                break;
            }
        }
    }
}

/* Output number k (k = 0, 1, ...) of SplitMix64 seeded with `seed`: the
 * generator's state after k+1 increments is seed + (k+1) * gamma, so the
 * state before the call that returns output k is seed + k * gamma. */
uint64_t orc_splitmix64_at(uint64_t seed, uint64_t k)
{
    uint64_t x = seed + k * 0x9e3779b97f4a7c15ULL;
    return orc_splitmix64_next(&x);
}

/* Random spacing (sec. 2.3: the same generator started from different
 * random states).  Stream g of the set starts at the state expanded, as for
 * a master seed, from output g of SplitMix64 seeded with `master`. */
void orc_random_spacing(uint64_t master, uint64_t first, uint64_t count, uint32_t *out)
{
    for (uint64_t i = 0; i < count; ++i)
        orc_seed_from_master(orc_splitmix64_at(master, first + i), out + 6 * i);
}

/* 1 when the state is a valid MRG32k3a state: each word below its modulus
 * and neither triple all zero (the all-zero triple is a fixed point). */
int orc_state_valid(const uint32_t s[6])
{
    if (s[0] >= ORC_M1 || s[1] >= ORC_M1 || s[2] >= ORC_M1) return 0;
    if (s[3] >= ORC_M2 || s[4] >= ORC_M2 || s[5] >= ORC_M2) return 0;
    if ((s[0] | s[1] | s[2]) == 0 || (s[3] | s[4] | s[5]) == 0) return 0;
    return 1;
}

/* ---------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC 2011), the counter-based  */
/* family the paper embeds beside MRG32k3a: ten rounds of a multiply-and-  */
/* xor bijection of a 128-bit counter under a 64-bit key.  Each round      */
/* multiplies counter words 0 and 2 by the two multipliers, keeps the low  */
/* halves as the new words 3 and 1, and xors the high halves with the      */
/* other two words and the round key into the new words 2 and 0.  The      */
/* round key starts at the key and moves by the two Weyl increments        */
/* between rounds.                                                         */
/* ---------------------------------------------------------------------- */
#define ORC_PHILOX_M0 0xD2511F53u
#define ORC_PHILOX_M1 0xCD9E8D57u
#define ORC_PHILOX_W0 0x9E3779B9u
#define ORC_PHILOX_W1 0xBB67AE85u

void orc_philox_constants(uint32_t out[4])
{
    out[0] = ORC_PHILOX_M0;
    out[1] = ORC_PHILOX_M1;
    out[2] = ORC_PHILOX_W0;
    out[3] = ORC_PHILOX_W1;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += ORC_PHILOX_W0;
            k1 += ORC_PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)ORC_PHILOX_M0 * c0;
        uint64_t p1 = (uint64_t)ORC_PHILOX_M1 * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* A Philox stream's 6 state words: (position lo, hi, stream id lo, hi, key lo,
 * hi).  Output number `position` is word position % 4 of the block with
 * counter (position / 4 as two words, stream id as two words). */
uint32_t orc_philox_next(uint32_t st[6])
{
    uint64_t pos = (uint64_t)st[0] | (uint64_t)st[1] << 32;
    uint64_t b = pos >> 2;
    uint32_t ctr[4] = {(uint32_t)b, (uint32_t)(b >> 32), st[2], st[3]};
    uint32_t key[2] = {st[4], st[5]};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    uint32_t z = w[pos & 3];
    pos += 1;
    st[0] = (uint32_t)pos;
    st[1] = (uint32_t)(pos >> 32);
    return z;
}

/* Conversions of a 32-bit word: odd multiples of 2^-24 from its top 23 bits
 * (binary32) and of 2^-33 from all 32 (binary64), both exact (24 and 33
 * significant bits) and inside (0, 1). */
float orc_philox_to_f32(uint32_t w) { return (float)(2u * (w >> 9) + 1u) * 0x1p-24f; }
double orc_philox_to_f64(uint32_t w) { return ((double)w * 2.0 + 1.0) * 0x1p-33; }

void orc_philox_fill(uint32_t *states, uint64_t S, uint64_t n, int dtype, int layout, void *out)
{
    for (uint64_t s = 0; s < S; ++s) {
        uint32_t *st = states + 6 * s;
        for (uint64_t k = 0; k < n; ++k) {
            uint32_t w = orc_philox_next(st);
            uint64_t idx = (layout == ORC_STREAM_MAJOR) ? s * n + k : k * S + s;
            if (dtype == ORC_U32)      ((uint32_t *)out)[idx] = w;
            else if (dtype == ORC_F32) ((float *)out)[idx] = orc_philox_to_f32(w);
            else                       ((double *)out)[idx] = orc_philox_to_f64(w);
        }
    }
}

/* Stream g of a Philox set under `key` starts at position 0 with id g. */
void orc_philox_streams(uint64_t key, uint64_t first, uint64_t count, uint32_t *out)
{
    for (uint64_t i = 0; i < count; ++i) {
        uint64_t g = first + i;
        uint32_t *st = out + 6 * i;
        st[0] = 0;
        st[1] = 0;
        st[2] = (uint32_t)g;
        st[3] = (uint32_t)(g >> 32);
        st[4] = (uint32_t)key;
        st[5] = (uint32_t)(key >> 32);
    }
}
