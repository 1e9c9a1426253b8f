// Host build of the library's device arithmetic (mrg_arith.hpp) for CPU
// tests: both formulations, stepped from a given state, so that the tests can
// compare them with the oracle on boundary inputs without a GPU.
#include <stdint.h>
#include "mrg_arith.hpp"

using namespace mrg;

extern "C" {

// n outputs (z' in [1, m1]) of the integer formulation from a lazy state
// w[6]; w is advanced (left lazy).
void shim_run_int(uint32_t *w, uint64_t n, uint32_t *out)
{
    uint32_t a0 = w[0], a1 = w[1], a2 = w[2], b0 = w[3], b1 = w[4], b2 = w[5];
    for (uint64_t k = 0; k < n; ++k) {
        const uint32_t p1 = next1(a0, a1), p2 = next2(b0, b2);
        a0 = a1; a1 = a2; a2 = p1;
        b0 = b1; b1 = b2; b2 = p2;
        out[k] = combine(p1, p2);
    }
    w[0] = a0; w[1] = a1; w[2] = a2; w[3] = b0; w[4] = b1; w[5] = b2;
}

// Same for the binary64 formulation from a canonical state; w receives the
// canonical state after n steps.  Also returns the f32/f64 conversions.
void shim_run_f64(uint32_t *w, uint64_t n, uint32_t *out, float *outf, double *outd)
{
    double a0 = w[0], a1 = w[1], a2 = w[2], b0 = w[3], b1 = w[4], b2 = w[5];
    for (uint64_t k = 0; k < n; ++k) {
        const double r1 = next1f(a0, a1), r2 = next2f(b0, b2);
        a0 = a1; a1 = a2; a2 = r1;
        b0 = b1; b1 = b2; b2 = r2;
        const double z = combinef(r1, r2);
        out[k] = (uint32_t)z;
        outf[k] = to_f32f(z);
        outd[k] = to_f64f(z);
    }
    w[0] = canonf(a0, M1D); w[1] = canonf(a1, M1D); w[2] = canonf(a2, M1D);
    w[3] = canonf(b0, M2D); w[4] = canonf(b1, M2D); w[5] = canonf(b2, M2D);
}

// Checked draws as the wave writer takes them: blocks of `block` values drawn
// with the three-operation combination while the high words of the new
// component-2 words are or-ed together; a block whose or comes out with the
// sign bit set is drawn again, exactly, from the state it started at.
// Returns the number of blocks drawn again; w as in shim_run_f64.
uint64_t shim_run_f64_checked(uint32_t *w, uint64_t n, uint64_t block, uint32_t *out)
{
    double a0 = w[0], a1 = w[1], a2 = w[2], b0 = w[3], b1 = w[4], b2 = w[5];
    uint64_t redrawn = 0;
    for (uint64_t k0 = 0; k0 < n; k0 += block) {
        const uint64_t k1 = k0 + block < n ? k0 + block : n;
        const double s[6] = {a0, a1, a2, b0, b1, b2};
        uint32_t neg = 0;
        for (uint64_t k = k0; k < k1; ++k) {
            const double r1 = next1f(a0, a1), r2 = next2f(b0, b2);
            a0 = a1; a1 = a2; a2 = r1;
            b0 = b1; b1 = b2; b2 = r2;
            neg |= hi_word(r2);
            out[k] = (uint32_t)combinef_nn(r1, r2);
        }
        if ((int32_t)neg < 0) {
            ++redrawn;
            double c0 = s[0], c1 = s[1], c2 = s[2], d0 = s[3], d1 = s[4], d2 = s[5];
            for (uint64_t k = k0; k < k1; ++k) {
                const double r1 = next1f(c0, c1), r2 = next2f(d0, d2);
                c0 = c1; c1 = c2; c2 = r1;
                d0 = d1; d1 = d2; d2 = r2;
                out[k] = (uint32_t)combinef(r1, r2);
            }
        }
    }
    w[0] = canonf(a0, M1D); w[1] = canonf(a1, M1D); w[2] = canonf(a2, M1D);
    w[3] = canonf(b0, M2D); w[4] = canonf(b1, M2D); w[5] = canonf(b2, M2D);
    return redrawn;
}

uint32_t shim_combine(uint32_t x1, uint32_t x2) { return combine(x1, x2); }
double shim_combinef_nn(double r1, double r2) { return combinef_nn(r1, r2); }
uint32_t shim_hi_word(double x) { return hi_word(x); }
double shim_combinef(double r1, double r2) { return combinef(r1, r2); }
double shim_next1f(double s0, double s1) { return next1f(s0, s1); }
double shim_next2f(double s3, double s5) { return next2f(s3, s5); }
uint32_t shim_canon1(uint32_t x) { return canon1(x); }
uint32_t shim_canon2(uint32_t x) { return canon2(x); }
uint32_t shim_canonf(double r, int comp) { return canonf(r, comp ? M2D : M1D); }
float shim_to_f32(uint32_t z) { return to_f32(z); }
double shim_to_f64(uint32_t z) { return to_f64(z); }
float shim_to_f32f(double z) { return to_f32f(z); }
uint32_t shim_dot3(int comp, const uint32_t *m, const uint32_t *x)
{
    return comp ? dot3_mod<C2>(m[0], m[1], m[2], x[0], x[1], x[2])
                : dot3_mod<C1>(m[0], m[1], m[2], x[0], x[1], x[2]);
}
}
