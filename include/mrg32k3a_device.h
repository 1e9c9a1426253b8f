/* Per-thread MRG32k3a streams inside user kernels (HIP, gfx950).
 *
 * The paper's generator object is built once per thread and drawn from with
 * next() inside the user's own kernel (sec. 5, Listing 1), the streams having
 * been placed on the host beforehand by jump-ahead (sec. 2.3, sec. 4.1).  This
 * header gives that mode on top of the library's stream sets: create a set
 * (mrg_streamset_create*), optionally jump it, read its device state planes
 * with mrg_streamset_states_ptr and its size with mrg_streamset_info, then in
 * a kernel
 *
 *     mrg::Stream<> s;
 *     s.load(planes, n_streams, i);      // stream i of the set
 *     float u = s.next_f32();            // ... as many draws as needed
 *     s.store(planes, n_streams, i);     // continue there next time
 *
 * Draws are bit-identical to mrg_fill's: value k of stream i here is value k
 * of row i of a stream-major fill started from the same state.  State words
 * live in registers; the planes hold word c of stream i at planes[c * n + i],
 * so loads and stores of consecutive streams by consecutive lanes coalesce.
 * The library's own kernels are built on the same types.
 *
 * Include path: this directory (the header also pulls in mrg_arith.hpp). */
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mrg_arith.hpp"

namespace mrg {

// Integer generator: lazy 32-bit words, v_mad_u64_u32 product-sums.  The
// multipliers live in VGPRs so that each v_mad_u64_u32 can take the constant
// addend K from an SGPR pair (one scalar operand per VOP3 instruction).
struct GenI {
    uint32_t a0, a1, a2, b0, b1, b2;  // lazy words, oldest first
    uint32_t m13, m12, m23, m21;      // multipliers held in VGPRs

    __device__ __forceinline__ void load(const uint32_t *w)
    {
        a0 = w[0]; a1 = w[1]; a2 = w[2]; b0 = w[3]; b1 = w[4]; b2 = w[5];
        m13 = A13N; m12 = A12; m23 = A23N; m21 = A21;
        asm volatile("" : "+v"(m13), "+v"(m12), "+v"(m23), "+v"(m21));
    }
    __device__ __forceinline__ void store(uint32_t *w) const
    {
        w[0] = canon1(a0); w[1] = canon1(a1); w[2] = canon1(a2);
        w[3] = canon2(b0); w[4] = canon2(b1); w[5] = canon2(b2);
    }
    __device__ __forceinline__ uint32_t step()
    {
        const uint32_t p1 = next1(a0, a1, m13, m12);
        const uint32_t p2 = next2(b0, b2, m23, m21);
        a0 = a1; a1 = a2; a2 = p1;
        b0 = b1; b1 = b2; b2 = p2;
        return combine(p1, p2);
    }
    __device__ __forceinline__ uint32_t next_u32() { return step(); }
    __device__ __forceinline__ float next_f32() { return to_f32(step()); }
    __device__ __forceinline__ double next_f64() { return to_f64(step()); }
    // Same values (the integer combination has no cheaper form to check).
    static constexpr bool kCheckedDraws = false;
    __device__ __forceinline__ uint32_t next_u32(uint32_t &) { return next_u32(); }
    __device__ __forceinline__ float next_f32(uint32_t &) { return next_f32(); }
    __device__ __forceinline__ double next_f64(uint32_t &) { return next_f64(); }
};

// Binary64 generator: near-canonical integer-valued doubles, five FP64 operations
// per component per step.
struct GenF {
    double a0, a1, a2, b0, b1, b2;

    __device__ __forceinline__ void load(const uint32_t *w)
    {
        a0 = w[0]; a1 = w[1]; a2 = w[2]; b0 = w[3]; b1 = w[4]; b2 = w[5];
    }
    __device__ __forceinline__ void store(uint32_t *w) const
    {
        w[0] = canonf(a0, M1D); w[1] = canonf(a1, M1D); w[2] = canonf(a2, M1D);
        w[3] = canonf(b0, M2D); w[4] = canonf(b1, M2D); w[5] = canonf(b2, M2D);
    }
    __device__ __forceinline__ double step()
    {
        const double r1 = next1f(a0, a1);
        const double r2 = next2f(b0, b2);
        a0 = a1; a1 = a2; a2 = r1;
        b0 = b1; b1 = b2; b2 = r2;
        return combinef(r1, r2);
    }
    __device__ __forceinline__ uint32_t next_u32() { return (uint32_t)step(); }
    __device__ __forceinline__ float next_f32() { return to_f32f(step()); }
    __device__ __forceinline__ double next_f64() { return to_f64f(step()); }

    // Checked draws: the state moves exactly as in step(), but the output
    // takes the three-operation combination combinef_nn, which is exact
    // unless the new component-2 word is negative (its residue within about
    // 5 of m2, some 5 times in 2^32 outputs).  That case sets the sign bit of
    // `neg`; a caller that sees it must replace the outputs drawn since it
    // cleared `neg` by ones drawn with next_*() from the same state.
    static constexpr bool kCheckedDraws = true;
    __device__ __forceinline__ double step_nn(uint32_t &neg)
    {
        const double r1 = next1f(a0, a1);
        const double r2 = next2f(b0, b2);
        a0 = a1; a1 = a2; a2 = r1;
        b0 = b1; b1 = b2; b2 = r2;
        // one v_or_b32 per draw, kept as written: left to itself the compiler
        // merges the ORs of an unrolled run of draws into 64-bit ORs at its
        // end, which keeps every component-2 word of the run live until then
        asm("v_or_b32 %0, %0, %1" : "+v"(neg) : "v"(__builtin_bit_cast(uint2, r2).y));
        return combinef_nn(r1, r2);
    }
    // Two checked draws (combined values za then zb) whose sign checks take
    // one v_or3_b32 between them, again kept as written.
    __device__ __forceinline__ void step2_nn(double &za, double &zb, uint32_t &neg)
    {
        const double r1a = next1f(a0, a1);
        const double r2a = next2f(b0, b2);
        a0 = a1; a1 = a2; a2 = r1a;
        b0 = b1; b1 = b2; b2 = r2a;
        const double r1b = next1f(a0, a1);
        const double r2b = next2f(b0, b2);
        a0 = a1; a1 = a2; a2 = r1b;
        b0 = b1; b1 = b2; b2 = r2b;
        asm("v_or3_b32 %0, %0, %1, %2"
            : "+v"(neg)
            : "v"(__builtin_bit_cast(uint2, r2a).y), "v"(__builtin_bit_cast(uint2, r2b).y));
        za = combinef_nn(r1a, r2a);
        zb = combinef_nn(r1b, r2b);
    }
    __device__ __forceinline__ uint32_t next_u32(uint32_t &neg) { return (uint32_t)step_nn(neg); }
    __device__ __forceinline__ float next_f32(uint32_t &neg) { return to_f32f(step_nn(neg)); }
    __device__ __forceinline__ double next_f64(uint32_t &neg) { return to_f64f(step_nn(neg)); }
};

__device__ __forceinline__ void load_state(const uint32_t *planes, uint64_t stride, uint64_t idx,
                                           uint32_t *w)
{
#pragma unroll
    for (int c = 0; c < 6; ++c) w[c] = planes[c * stride + idx];
}

__device__ __forceinline__ void store_state(uint32_t *planes, uint64_t stride, uint64_t idx,
                                            const uint32_t *w)
{
#pragma unroll
    for (int c = 0; c < 6; ++c) planes[c * stride + idx] = w[c];
}

// Windowed jump tables (mrg_streamset_tables_ptr): T[c][w][d] = A_c^(d * 16^w)
// mod m_c, row-major 3x3 uint32, c in {0,1}, w in [0, 48), d in [0, 16)
// (d = 0: identity), so any exponent below 2^192 is at most 48 products per
// component (sec. 2.3 jump-ahead).
constexpr int kTableWindows = 48;
constexpr int kTableWindowWords = 16 * 9;

// Digit w (4 bits) of a 192-bit exponent given as 3 little-endian words.
__device__ __forceinline__ uint32_t exp_digit(uint64_t e0, uint64_t e1, uint64_t e2, int w)
{
    const uint64_t word = w < 16 ? e0 : (w < 32 ? e1 : e2);
    return (uint32_t)(word >> (4 * (w & 15))) & 15u;
}

// One past the highest window holding a nonzero digit (0 for e = 0).
__device__ __forceinline__ int top_window(uint64_t e0, uint64_t e1, uint64_t e2)
{
    if (e2) return 32 + (67 - __clzll((long long)e2)) / 4;
    if (e1) return 16 + (67 - __clzll((long long)e1)) / 4;
    if (e0) return (67 - __clzll((long long)e0)) / 4;
    return 0;
}

// st <- A^e st with the tables read from global memory (L2-resident), over
// windows [w_lo, w_hi).  Windows whose digit is zero in every lane are
// skipped, and the loop ends after the wave's highest nonzero digit; when e
// is the same in every lane the table reads are uniform.
__device__ __forceinline__ void jump_global(const uint32_t *__restrict__ table, uint64_t e0,
                                            uint64_t e1, uint64_t e2, int w_lo, int w_hi,
                                            uint32_t *st)
{
    const int top = top_window(e0, e1, e2);
#pragma unroll 1
    for (int w = w_lo; w < w_hi; ++w) {
        if (!__any(w < top)) break;
        const uint32_t d = exp_digit(e0, e1, e2, w);
        if (!__any(d != 0u)) continue;
        if (d == 0u) continue;  // this lane's identity (exec-masked)
        matvec3<C1>(table + ((0 * kTableWindows + w) * 16 + d) * 9, st[0], st[1], st[2]);
        matvec3<C2>(table + ((1 * kTableWindows + w) * 16 + d) * 9, st[3], st[4], st[5]);
    }
}

// One stream drawn by one thread.  G = GenF (binary64 words, the default) or
// GenI (32-bit integer words).
template <class G = GenF>
struct Stream {
    G g;

    // Stream i of a set whose six state planes of n_streams words start at planes.
    __device__ __forceinline__ void load(const uint32_t *planes, uint64_t n_streams, uint64_t i)
    {
        uint32_t w[6];
        load_state(planes, n_streams, i, w);
        g.load(w);
    }
    // Write the state back (canonical words), e.g. to continue in a later launch.
    __device__ __forceinline__ void store(uint32_t *planes, uint64_t n_streams, uint64_t i) const
    {
        uint32_t w[6];
        g.store(w);
        store_state(planes, n_streams, i, w);
    }
    // Move e = e0 + e1 * 2^64 + e2 * 2^128 values ahead (tables: the set's
    // device jump tables).  Cheapest when e is the same in the whole wave.
    __device__ __forceinline__ void jump(const uint32_t *tables, uint64_t e0, uint64_t e1 = 0,
                                         uint64_t e2 = 0)
    {
        uint32_t w[6];
        g.store(w);
        jump_global(tables, e0, e1, e2, 0, kTableWindows, w);
        g.load(w);
    }
    // Move to substream j of the current position: j * 2^76 values ahead (sec. 4.1).
    __device__ __forceinline__ void substream(const uint32_t *tables, uint64_t j)
    {
        jump(tables, 0, j << 12, j >> 52);
    }
    // The next value as uint32 in [1, m1], as binary32 in (0, 1) or as binary64 in (0, 1).
    __device__ __forceinline__ uint32_t next_u32() { return g.next_u32(); }
    __device__ __forceinline__ float next_f32() { return g.next_f32(); }
    __device__ __forceinline__ double next_f64() { return g.next_f64(); }
};

}  // namespace mrg
