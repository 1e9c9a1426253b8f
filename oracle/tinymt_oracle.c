/*
 * TinyMT32 CPU oracle -- TEST INFRASTRUCTURE ONLY (built into the same
 * library as the MRG32k3a oracle; the same rules apply: only the tests, the
 * smoke check and the benchmark's CPU baseline may load it, and it shares
 * no code, header, table or constant generator with the GPU library).
 *
 * Method (Passerat-Palmbach & Hill, HPCS 2012, sec. 4.2 "TinyMT"): TinyMT
 * is a small Mersenne-Twister-family generator with a 127-bit state and a
 * period of 2^127 - 1, whose independent streams come from
 * parameterisation (each parameter set from Dynamic Creator is its own
 * generator).  The paper's hybrid shares one parameter set among all the
 * threads of a block and gives each thread a sub-stream of that generator
 * by sequence splitting: the sequence is cut into equal chunks whose first
 * states go to the threads by their identifier.  The generator itself is
 * the one its authors published (Saito & Matsumoto, TinyMT, 2011), cited by
 * the paper; the paper prints neither its recursion nor parameters.
 *
 * Everything here is written out plainly:
 *  - the state transition and the tempering of TinyMT32 (state words s0..s3,
 *    bit 31 of s0 outside the 127-bit state; parameters mat1, mat2, tmat);
 *  - the published seeding from a 32-bit seed;
 *  - polynomials over GF(2) as bit arrays in 64-bit words (coefficient i is
 *    bit i % 64 of word i / 64), with schoolbook multiplication and
 *    reduction;
 *  - the characteristic polynomial of a parameter set from the
 *    Berlekamp-Massey algorithm run on a linear output bit of the state;
 *  - Rabin's irreducibility test for a prime degree n: f is irreducible
 *    exactly when x^(2^n) = x mod f and f has no root in GF(2); for n = 127
 *    (a Mersenne exponent, 2^127 - 1 prime) an irreducible characteristic
 *    polynomial is primitive, so every nonzero state has period 2^127 - 1;
 *  - jumps by polynomial arithmetic: with g(x) = x^(J-1) mod phi(x), the
 *    state J steps ahead is one transition applied to g(T) s (Horner's
 *    rule), T the transition (the extra transition clears the one bit the
 *    127-dimensional arithmetic does not determine).
 *
 * Readings of points neither paper fixes (also listed in the design notes):
 *  - a parameter set is accepted when its characteristic polynomial has
 *    degree 127 and is irreducible; candidates (mat1, mat2, tmat) are drawn
 *    from SplitMix64 seeded with master_seed + 1 (candidate c: outputs 2c
 *    and 2c+1; mat1, mat2 the low and high half of the first, tmat the low
 *    half of the second); parameter set p of a stream set is the p-th
 *    accepted candidate.  Dynamic Creator's further selection of the
 *    tempering parameter for equidistribution is not made;
 *  - the base status of parameter set p is the published seeding from the
 *    32-bit seed = low half of SplitMix64 output p of master_seed;
 *  - thread (sub-stream) j of a parameter set starts j * 2^64 outputs past
 *    the base status;
 *  - uint32 outputs are the tempered words; FP32 (2 * (w >> 9) + 1) * 2^-24
 *    and FP64 (2w + 1) * 2^-33, as for the counter-based generator.
 *
 * Parity unpinned: no known-answer output of TinyMT32 is available here, so
 * the transition, tempering and seeding rest on their written definition;
 * the pins cover linearity, the period, Berlekamp-Massey, the
 * irreducibility test and jumps against brute-force stepping.
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>

#define TMT_MASK 0x7fffffffu
#define TMT_SH0 1
#define TMT_SH1 10
#define TMT_SH8 8

/* ---------------------------------------------------------------------- */
/* The generator                                                           */
/* ---------------------------------------------------------------------- */
/* One transition of the state s under parameters p = (mat1, mat2, tmat). */
void orc_tmt_next(uint32_t s[4], const uint32_t p[3])
{
    uint32_t x = (s[0] & TMT_MASK) ^ s[1] ^ s[2];
    uint32_t y = s[3];
    x ^= x << TMT_SH0;
    y ^= (y >> TMT_SH0) ^ x;
    uint32_t n0 = s[1];
    uint32_t n1 = s[2];
    uint32_t n2 = x ^ (y << TMT_SH1);
    uint32_t n3 = y;
    if (y & 1u) {
        n1 ^= p[0];
        n2 ^= p[1];
    }
    s[0] = n0; s[1] = n1; s[2] = n2; s[3] = n3;
}

/* The output word of a state (tempering; the addition makes it nonlinear). */
uint32_t orc_tmt_temper(const uint32_t s[4], const uint32_t p[3])
{
    uint32_t t1 = s[0] + (s[2] >> TMT_SH8);
    uint32_t t0 = s[3] ^ t1;
    if (t1 & 1u) t0 ^= p[2];
    return t0;
}

/* Output number 0 comes from the first transition. */
uint32_t orc_tmt_draw(uint32_t s[4], const uint32_t p[3])
{
    orc_tmt_next(s, p);
    return orc_tmt_temper(s, p);
}

/* Published seeding from a 32-bit seed. */
void orc_tmt_init(uint32_t seed, const uint32_t p[3], uint32_t s[4])
{
    s[0] = seed; s[1] = p[0]; s[2] = p[1]; s[3] = p[2];
    for (uint32_t i = 1; i < 8; ++i) {
        uint32_t prev = s[(i - 1) & 3];
        s[i & 3] ^= i + 1812433253u * (prev ^ (prev >> 30));
    }
    if ((s[0] & TMT_MASK) == 0 && s[1] == 0 && s[2] == 0 && s[3] == 0) {
        s[0] = 'T'; s[1] = 'I'; s[2] = 'N'; s[3] = 'Y';
    }
    for (int i = 0; i < 8; ++i) orc_tmt_next(s, p);
}

/* ---------------------------------------------------------------------- */
/* Polynomials over GF(2), degree < 256 (4 words)                          */
/* ---------------------------------------------------------------------- */
#define PW 4
typedef struct { uint64_t w[PW]; } poly;

static int pbit(const poly *a, int i) { return (int)((a->w[i >> 6] >> (i & 63)) & 1u); }
static void pset(poly *a, int i) { a->w[i >> 6] |= (uint64_t)1 << (i & 63); }
static void pflip(poly *a, int i) { a->w[i >> 6] ^= (uint64_t)1 << (i & 63); }

static int pdeg(const poly *a)
{
    for (int i = 64 * PW - 1; i >= 0; --i)
        if (pbit(a, i)) return i;
    return -1;
}

/* r ^= a * x^sh (terms shifted past degree 255 are dropped; a's terms
 * stay below 128 wherever this is used, so none are). */
static void pxor_shifted(poly *r, const poly *a, int sh)
{
    int ws = sh >> 6, bs = sh & 63;
    for (int i = PW - 1; i >= ws; --i) {
        uint64_t v = a->w[i - ws] << bs;
        if (bs && i - ws - 1 >= 0) v |= a->w[i - ws - 1] >> (64 - bs);
        r->w[i] ^= v;
    }
}

/* a mod f (f of degree d >= 1), cancelling the top coefficient of a with
 * f * x^(i-d) from the top down. */
static poly pmod(poly a, const poly *f)
{
    int d = pdeg(f);
    for (int i = 64 * PW - 1; i >= d; --i)
        if (pbit(&a, i)) pxor_shifted(&a, f, i - d);
    return a;
}

/* a * b mod f, a and b of degree below deg f <= 127: the sum of b * x^i
 * over the terms x^i of a, then reduced. */
static poly pmulmod(const poly *a, const poly *b, const poly *f)
{
    poly r;
    memset(&r, 0, sizeof r);
    for (int i = 0; i < 128; ++i)
        if (pbit(a, i)) pxor_shifted(&r, b, i);
    return pmod(r, f);
}

/* x^e mod f, e = e[0] + e[1] * 2^64, by square-and-multiply from the top bit. */
static poly pxpow(const uint64_t e[2], const poly *f)
{
    poly r, x;
    memset(&r, 0, sizeof r);
    memset(&x, 0, sizeof x);
    pset(&r, 0);
    pset(&x, 1);
    x = pmod(x, f);
    for (int b = 127; b >= 0; --b) {
        r = pmulmod(&r, &r, f);
        if ((e[b >> 6] >> (b & 63)) & 1u) r = pmulmod(&r, &x, f);
    }
    return r;
}

/* The polynomial f (coefficients as 4 words) is irreducible, for a prime
 * degree n = deg f: x^(2^n) = x mod f, f(0) = 1 and f(1) = 1 (Rabin). */
int orc_gf2_irreducible_prime_degree(const uint64_t fw[4])
{
    poly f;
    memcpy(f.w, fw, sizeof f.w);
    int n = pdeg(&f);
    if (n < 1) return 0;
    if (!pbit(&f, 0)) return 0;          /* root 0 */
    int ones = 0;
    for (int i = 0; i <= n; ++i) ones += pbit(&f, i);
    if (!(ones & 1)) return 0;           /* root 1 */
    poly t;
    memset(&t, 0, sizeof t);
    pset(&t, 1);
    t = pmod(t, &f);
    for (int i = 0; i < n; ++i) t = pmulmod(&t, &t, &f);
    poly x;
    memset(&x, 0, sizeof x);
    pset(&x, 1);
    x = pmod(x, &f);
    return memcmp(t.w, x.w, sizeof t.w) == 0;
}

/* Berlekamp-Massey over GF(2): the shortest connection polynomial C with
 * sum_{i=0..L} C_i a_{k-i} = 0 for k = L .. N-1 (C_0 = 1).  Returns L and
 * writes C (bit i = C_i) to c; bits a[0..N-1], N <= 255. */
int orc_gf2_berlekamp_massey(const uint8_t *a, int N, uint64_t cw[4])
{
    poly C, B;
    memset(&C, 0, sizeof C);
    memset(&B, 0, sizeof B);
    pset(&C, 0);
    pset(&B, 0);
    int L = 0, m = 1;
    for (int k = 0; k < N; ++k) {
        int d = a[k];
        for (int i = 1; i <= L; ++i) d ^= pbit(&C, i) & a[k - i];
        if (!d) {
            ++m;
            continue;
        }
        poly T = C;
        pxor_shifted(&C, &B, m);
        if (2 * L <= k) {
            L = k + 1 - L;
            B = T;
            m = 1;
        } else {
            ++m;
        }
    }
    memcpy(cw, C.w, sizeof C.w);
    return L;
}

/* Characteristic polynomial of a parameter set's transition: the minimal
 * polynomial of the sequence of bit 0 of s3 (a linear function of the
 * state), from 254 terms.  phi(x) = x^L C(1/x).  Returns L (127 when the
 * sequence is as long as the state allows). */
int orc_tmt_charpoly(const uint32_t p[3], uint64_t phi[4])
{
    uint32_t s[4] = {0x12345678u, 0x9abcdef0u, 0x0fedcba9u, 0x87654321u};
    uint8_t a[254];
    for (int k = 0; k < 254; ++k) {
        orc_tmt_next(s, p);
        a[k] = (uint8_t)(s[3] & 1u);
    }
    uint64_t cw[4];
    int L = orc_gf2_berlekamp_massey(a, 254, cw);
    poly C, F;
    memcpy(C.w, cw, sizeof C.w);
    memset(&F, 0, sizeof F);
    for (int i = 0; i <= L; ++i)
        if (pbit(&C, i)) pset(&F, L - i);
    memcpy(phi, F.w, sizeof F.w);
    return L;
}

/* 1 when the parameter set's transition has an irreducible characteristic
 * polynomial of degree 127 (period 2^127 - 1). */
int orc_tmt_params_ok(const uint32_t p[3])
{
    uint64_t phi[4];
    if (orc_tmt_charpoly(p, phi) != 127) return 0;
    return orc_gf2_irreducible_prime_degree(phi);
}

/* ---------------------------------------------------------------------- */
/* Jumps                                                                   */
/* ---------------------------------------------------------------------- */
/* s <- T^e s for e = e[0] + e[1] * 2^64, phi the parameter set's
 * characteristic polynomial. */
void orc_tmt_jump(uint32_t s[4], const uint32_t p[3], const uint64_t phiw[4], const uint64_t e[2])
{
    if (e[0] == 0 && e[1] == 0) return;
    poly phi;
    memcpy(phi.w, phiw, sizeof phi.w);
    uint64_t em1[2] = {e[0] - 1, e[1] - (e[0] == 0 ? 1u : 0u)};
    poly g = pxpow(em1, &phi);
    uint32_t acc[4] = {0, 0, 0, 0};
    for (int i = pdeg(&phi) - 1; i >= 0; --i) {
        orc_tmt_next(acc, p);
        if (pbit(&g, i))
            for (int k = 0; k < 4; ++k) acc[k] ^= s[k];
    }
    orc_tmt_next(acc, p);
    memcpy(s, acc, 4 * sizeof(uint32_t));
}

/* s <- T^k s by stepping. */
void orc_tmt_skip(uint32_t s[4], const uint32_t p[3], uint64_t k)
{
    for (uint64_t i = 0; i < k; ++i) orc_tmt_next(s, p);
}

/* ---------------------------------------------------------------------- */
/* Parameter sets and stream sets                                          */
/* ---------------------------------------------------------------------- */
extern uint64_t orc_splitmix64_at(uint64_t seed, uint64_t k);

/* Candidate c of the search seeded by master (see the readings above). */
void orc_tmt_candidate(uint64_t master, uint64_t c, uint32_t p[3])
{
    uint64_t a = orc_splitmix64_at(master + 1, 2 * c);
    uint64_t b = orc_splitmix64_at(master + 1, 2 * c + 1);
    p[0] = (uint32_t)a;
    p[1] = (uint32_t)(a >> 32);
    p[2] = (uint32_t)b;
}

/* Parameter sets 0 .. count-1 of master's search: out[3 * i ..] and their
 * candidate numbers (cand may be NULL). */
void orc_tmt_search(uint64_t master, uint64_t count, uint32_t *out, uint64_t *cand)
{
    uint64_t c = 0;
    for (uint64_t i = 0; i < count; ++i) {
        for (;;) {
            uint32_t p[3];
            orc_tmt_candidate(master, c, p);
            ++c;
            if (orc_tmt_params_ok(p)) {
                memcpy(out + 3 * i, p, sizeof p);
                if (cand) cand[i] = c - 1;
                break;
            }
        }
    }
}

/* Start states of streams first .. first+count-1 of a TinyMT stream set:
 * global stream g uses parameter set q = g / per_param (params[q - q0], the
 * caller passing sets q0 ..) and is sub-stream j = g % per_param of it,
 * j * 2^64 outputs past the base status seeded from the low half of
 * SplitMix64 output q of master.  out[6 * i ..] = (s0, s1, s2, s3, q, 0). */
void orc_tmt_streams(uint64_t master, uint64_t per_param, uint64_t first, uint64_t count,
                     const uint32_t *params, uint64_t q0, uint32_t *out)
{
    uint64_t phi[4], phi_q = UINT64_MAX;
    for (uint64_t i = 0; i < count; ++i) {
        uint64_t g = first + i, q = g / per_param, j = g % per_param;
        const uint32_t *p = params + 3 * (q - q0);
        if (q != phi_q) {
            orc_tmt_charpoly(p, phi);
            phi_q = q;
        }
        uint32_t s[4];
        orc_tmt_init((uint32_t)orc_splitmix64_at(master, q), p, s);
        uint64_t e[2] = {0, j};
        orc_tmt_jump(s, p, phi, e);
        uint32_t *o = out + 6 * i;
        memcpy(o, s, sizeof s);
        o[4] = (uint32_t)q;
        o[5] = 0;
    }
}

float orc_tmt_to_f32(uint32_t w) { return (float)(2u * (w >> 9) + 1u) * 0x1p-24f; }
double orc_tmt_to_f64(uint32_t w) { return ((double)w * 2.0 + 1.0) * 0x1p-33; }

/* n outputs of each of S streams (states [S][6] as orc_tmt_streams writes
 * them, advanced in place; word 4 is the parameter set, params[3 * (q -
 * q0)]), stream-major out[s * n + k] or interleaved out[k * S + s]. */
void orc_tmt_fill(uint32_t *states, uint64_t S, uint64_t n, int dtype, int layout,
                  const uint32_t *params, uint64_t q0, void *out)
{
    for (uint64_t s = 0; s < S; ++s) {
        uint32_t *st = states + 6 * s;
        const uint32_t *p = params + 3 * (st[4] - q0);
        for (uint64_t k = 0; k < n; ++k) {
            uint32_t w = orc_tmt_draw(st, p);
            uint64_t idx = layout == 0 ? s * n + k : k * S + s;
            if (dtype == 0)      ((uint32_t *)out)[idx] = w;
            else if (dtype == 1) ((float *)out)[idx] = orc_tmt_to_f32(w);
            else                 ((double *)out)[idx] = orc_tmt_to_f64(w);
        }
    }
}
