// Device building blocks shared by the fill kernels and the persistent batch
// kernel: the two generator engines, 16-byte output packing, state planes,
// jump-table application, workgroup placement on the XCDs, and the LDS-staged
// writers
//   rows_fill       -- one stream per lane (rows of the LDS tile are streams);
//   rows_fill_short -- one stream per lane, rows shorter than a line, the
//                      wave's rows copied out as one block;
//   wave_fill       -- GL lanes per stream (64/GL streams per wave), member g
//                      owning consecutive L-value segments, so that each flush
//                      writes whole 128-byte lines.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"
#include "mrg32k3a_device.h"

namespace mrg {

template <int DT> struct Elem;
template <> struct Elem<0> { static constexpr int size = 4; };
template <> struct Elem<1> { static constexpr int size = 4; };
template <> struct Elem<2> { static constexpr int size = 8; };

// 16 bytes of output: 4 uint32 / 4 float / 2 double values.
template <int DT, class G>
__device__ __forceinline__ uint4 gen16(G &g)
{
    uint4 v;
    if constexpr (DT == 0) {
        v.x = g.next_u32(); v.y = g.next_u32(); v.z = g.next_u32(); v.w = g.next_u32();
    } else if constexpr (DT == 1) {
        v.x = __float_as_uint(g.next_f32());
        v.y = __float_as_uint(g.next_f32());
        v.z = __float_as_uint(g.next_f32());
        v.w = __float_as_uint(g.next_f32());
    } else {
        const uint64_t u0 = (uint64_t)__double_as_longlong(g.next_f64());
        const uint64_t u1 = (uint64_t)__double_as_longlong(g.next_f64());
        v.x = (uint32_t)u0; v.y = (uint32_t)(u0 >> 32);
        v.z = (uint32_t)u1; v.w = (uint32_t)(u1 >> 32);
    }
    return v;
}

// The same 16 bytes from checked draws (G::kCheckedDraws), taken in pairs
// (one sign check instruction per pair): exact unless the sign bit of `neg`
// comes out set (see GenF).
template <int DT, class G>
__device__ __forceinline__ uint4 gen16(G &g, uint32_t &neg)
{
    uint4 v;
    double z0, z1;
    g.step2_nn(z0, z1, neg);
    if constexpr (DT == 2) {
        const uint64_t u0 = (uint64_t)__double_as_longlong(to_f64f(z0));
        const uint64_t u1 = (uint64_t)__double_as_longlong(to_f64f(z1));
        v.x = (uint32_t)u0; v.y = (uint32_t)(u0 >> 32);
        v.z = (uint32_t)u1; v.w = (uint32_t)(u1 >> 32);
    } else {
        double z2, z3;
        g.step2_nn(z2, z3, neg);
        if constexpr (DT == 0) {
            v.x = (uint32_t)z0; v.y = (uint32_t)z1; v.z = (uint32_t)z2; v.w = (uint32_t)z3;
        } else {
            v.x = __float_as_uint(to_f32f(z0));
            v.y = __float_as_uint(to_f32f(z1));
            v.z = __float_as_uint(to_f32f(z2));
            v.w = __float_as_uint(to_f32f(z3));
        }
    }
    return v;
}

template <int DT, class G>
__device__ __forceinline__ void put1(unsigned char *p, G &g)
{
    if constexpr (DT == 0) *(uint32_t *)p = g.next_u32();
    else if constexpr (DT == 1) *(float *)p = g.next_f32();
    else *(double *)p = g.next_f64();
}

// 16-byte store at base + off where base is the same for the whole wave: the
// base goes into a raw buffer descriptor in scalar registers (word 3 0x20000:
// 32-bit data format, as gfx9 raw buffers take it), so a lane spends no vector
// instruction on its 64-bit address.  Offsets at or past span are dropped.
// AUX is the instruction's cache-policy field (0: the default write-back).
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t uniform_rsrc(const unsigned char *base,
                                                              uint32_t span)
{
    const uint64_t b = (uint64_t)base;
    const uint64_t bu = (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b) |
                        (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32)) << 32;
    return __builtin_amdgcn_make_buffer_rsrc((void *)bu, 0, (int)span, 0x00020000);
}

template <int AUX = 0>
__device__ __forceinline__ void store16_uniform(const unsigned char *base, uint32_t off,
                                                uint32_t span, uint4 v)
{
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4_t, v), uniform_rsrc(base, span),
                                           off, 0, AUX);
}

// 16-byte store at soff + voff bytes past the base of descriptor r (soff
// wave-uniform, voff per lane).
template <int AUX = 0>
__device__ __forceinline__ void store16_rsrc(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff,
                                             uint4 v)
{
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4_t, v), r, voff, soff, AUX);
}

template <int ES>
__device__ __forceinline__ void copy_elem(unsigned char *dst, const unsigned char *src)
{
    if constexpr (ES == 4) *(uint32_t *)dst = *(const uint32_t *)src;
    else *(uint64_t *)dst = *(const uint64_t *)src;
}

// ---------------------------------------------------------------------------
// rows_fill: one wave, lane r generates n values of its own stream (rows
// r < nrows are written; row r starts at out0 + r * row_stride, which must be
// ES-aligned).  Each row is cut into a head (the values before its first
// 128-byte line boundary), full tiles of TB bytes, and a tail.  Every part
// goes through the lane's LDS row: a full tile is written back as 16-byte
// chunks, TB/16 lanes per row, so one store instruction covers 64*16/TB rows x
// TB contiguous, line-aligned bytes; head and tail (fewer than 128 / ES and
// TB / ES values) are written back as dwords, TB/4 lanes per row.  The row pitch TB+16
// keeps both the b128 writes (lanes on different rows) and the reads (lanes
// along a row) free of bank conflicts.  `lds` holds 64 * (TB + 16) bytes; the
// caller's workgroup is this one wave.
// ---------------------------------------------------------------------------
template <int ES>
__device__ __forceinline__ uint64_t head_values(const unsigned char *row, uint64_t n)
{
    const uint64_t h = ((128u - ((uint32_t)(uintptr_t)row & 127u)) & 127u) / ES;
    return h < n ? h : n;
}

// Write back a partial part of every row from LDS: row r (< nrows) gets the
// first bytes_of(r) bytes of its LDS row at row + off_of(r), as dwords, TB/4
// lanes per row.  part(r, row, &off, &bytes) describes row r.
template <int TB, class Part>
__device__ __forceinline__ void rows_flush_part(const unsigned char *lds, int lane, uint64_t nrows,
                                                unsigned char *out0, uint64_t row_stride,
                                                const Part &part)
{
    constexpr int RS = TB + 16, DPR = TB / 4, RPD = 64 / DPR;
    const int rsub = lane / DPR;
    const uint32_t dl = (lane % DPR) * 4;
#pragma unroll 1
    for (int r = rsub; r < 64; r += RPD) {
        if ((uint64_t)r >= nrows) break;
        unsigned char *row = out0 + (uint64_t)r * row_stride;
        uint64_t off, bytes;
        part(row, off, bytes);
        if (dl < bytes) *(uint32_t *)(row + off + dl) = *(const uint32_t *)(lds + r * RS + dl);
    }
}

template <int DT, int TB, class G, bool READ_ALL = true>
__device__ __forceinline__ void rows_fill(G &g, unsigned char *lds, int lane, uint64_t nrows,
                                          unsigned char *out0, uint64_t row_stride, uint64_t n)
{
    constexpr int ES = Elem<DT>::size;
    constexpr int TV = TB / ES;      // values per row per tile
    constexpr int RS = TB + 16;      // LDS row pitch (bytes)
    constexpr int LPR = TB / 16;     // lanes per row when flushing
    constexpr int RPI = 64 / LPR;    // rows per flush instruction
    constexpr int NJ = 64 / RPI;     // flush instructions per tile

    const bool active = (uint64_t)lane < nrows;
    unsigned char *myrow = out0 + (uint64_t)lane * row_stride;
    const uint64_t hd = active ? head_values<ES>(myrow, n) : 0;
    const uint64_t nfull = (n - hd) / TV;  // n / TV or one less

    unsigned char *my_lds = lds + lane * RS;
    // head (only rows that start off a line boundary have one)
    if (__any(hd != 0)) {
        for (uint64_t c = 0; __any(c < hd); ++c)
            if (c < hd) put1<DT>(my_lds + c * ES, g);
        __syncthreads();
        rows_flush_part<TB>(lds, lane, nrows, out0, row_stride,
                            [n](const unsigned char *row, uint64_t &off, uint64_t &bytes) {
                                off = 0;
                                bytes = head_values<ES>(row, n) * ES;
                            });
        __syncthreads();
    }

    // the flush rows of this lane: their aligned tile base and tile count
    const int chunk = lane % LPR;
    unsigned char *rowp[NJ];
    uint32_t short_mask = 0;  // bit j: row j has n / TV - 1 full tiles
    bool rowa[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int r = lane / LPR + RPI * j;
        unsigned char *row = out0 + (uint64_t)r * row_stride;
        const uint64_t h = head_values<ES>(row, n);
        rowa[j] = (uint64_t)r < nrows;
        rowp[j] = row + h * ES + chunk * 16;
        if ((n - h) / TV < n / TV) short_mask |= 1u << j;
    }

    const uint64_t ntiles = n / TV;
    for (uint64_t t = 0; t < ntiles; ++t) {
        if (t < nfull) {
            if constexpr (G::kCheckedDraws) {
                // checked draws; the whole tile again, exactly, when a lane's
                // check fails (rare: the same rule as in wave_fill)
                const G saved = g;
                uint32_t neg = 0;
#pragma unroll
                for (int c = 0; c < TB / 16; ++c) *(uint4 *)(my_lds + c * 16) = gen16<DT>(g, neg);
                if (__any((int32_t)neg < 0)) {
                    g = saved;
#pragma unroll 1
                    for (int c = 0; c < TB / 16; ++c) *(uint4 *)(my_lds + c * 16) = gen16<DT>(g);
                }
            } else {
#pragma unroll
                for (int c = 0; c < TB / 16; ++c) *(uint4 *)(my_lds + c * 16) = gen16<DT>(g);
            }
        }
        __syncthreads();
        const uint64_t off = t * TB;
        const bool last = t + 1 == ntiles;
        if (READ_ALL) {
            // all LDS reads first, one wait, then the stores
            uint4 v[NJ];
#pragma unroll
            for (int j = 0; j < NJ; ++j)
                v[j] = *(const uint4 *)(lds + (lane / LPR + RPI * j) * RS + chunk * 16);
#pragma unroll
            for (int j = 0; j < NJ; ++j)
                if (rowa[j] && !(last && ((short_mask >> j) & 1u))) *(uint4 *)(rowp[j] + off) = v[j];
        } else {
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const uint4 v = *(const uint4 *)(lds + (lane / LPR + RPI * j) * RS + chunk * 16);
                if (rowa[j] && !(last && ((short_mask >> j) & 1u))) *(uint4 *)(rowp[j] + off) = v;
            }
        }
        __syncthreads();
    }

    // tail
    const uint64_t tail = active ? n - hd - nfull * TV : 0;
    if (__any(tail != 0)) {
        for (uint64_t c = 0; __any(c < tail); ++c)
            if (c < tail) put1<DT>(my_lds + c * ES, g);
        __syncthreads();
        rows_flush_part<TB>(lds, lane, nrows, out0, row_stride,
                            [n](const unsigned char *row, uint64_t &off, uint64_t &bytes) {
                                const uint64_t h = head_values<ES>(row, n);
                                const uint64_t t0 = h + (n - h) / TV * TV;
                                off = t0 * ES;
                                bytes = (n - t0) * ES;
                            });
        __syncthreads();
    }
}

// rows_fill_carry: as rows_fill (one stream per lane, row r < nrows of n
// values at out0 + r * n * ES: contiguous rows, ES-aligned, at least one line
// long), for rows off their lines.  Every lane draws the same number of
// values in every step whatever its row's alignment, and each line shared by
// two rows of the wave is written once, whole.  Row r is written through
// windows of TB bytes aligned to 128-byte lines: window k covers the row's
// bytes [k*TB - o, k*TB - o + TB), o = the row's offset past its first line.
// Step k draws the row's values [k*TV, k*TV + TV) into the lane's LDS row at
// byte o (filling window k from o on and spilling o bytes into window k+1);
// the wave then writes the lines of window k that lie wholly in their row,
// and the spilled bytes move to the front of the LDS row for the next
// window.  A row's first line (when o > 0) and last line (when the row ends
// off a line) are kept in registers instead; at the end each first line is
// written whole from the two rows that share it (the wave's first and last
// lines only in part: their other bytes belong to the neighbouring waves).
// With checked draws (GenF) a step whose sign check fails in some lane is
// drawn again exactly from the state saved before it.  `lds` holds
// 64 * (TB + 160) bytes.
//
// LDS banks: lane r stages its row at byte r * RS + o_r, o_r = r * nb mod 128
// (plus a constant), so one write step puts lane r on dword bank
// r * (RS + nb) / 4 mod 32: with a pitch of TB + 144 bytes and rows of
// nb / 4 = 4 mod 8 dwords that stride is a multiple of 8 dwords and up to all
// 32 lanes hit one bank (rows of 1500 or 5500 uint32 ran at 1.8-2.0 TB/s);
// such rows take a pitch of TB + 160.  Rows a multiple of 16 bytes long on a
// 16-byte aligned base are staged with 16-byte writes, one per four values,
// which with the pitch chosen so go to distinct banks; other rows with dword
// writes (their stride is then odd or twice odd: at most two-way).
template <int DT, int TB, class G, bool WIDE>
__device__ __forceinline__ void rows_fill_carry_w(G &g, unsigned char *lds, int lane, uint64_t nrows,
                                                  unsigned char *out0, uint64_t n)
{
    constexpr int ES = Elem<DT>::size;
    constexpr int TV = TB / ES;      // values per step
    constexpr int LPR = TB / 16;     // lanes per row when writing a window
    constexpr int RPI = 64 / LPR;    // rows per store instruction
    constexpr int NJ = 64 / RPI;     // store instructions per window
    static_assert(TB % 128 == 0 && TB <= 256, "windows of whole lines");

    const uint64_t nb = n * ES;      // bytes per row
    // LDS row: window + spill (< 128 bytes) + pad, its pitch by the row length
    const uint32_t RS = (nb / 4) % 8 == 4 ? TB + 160 : TB + 144;
    unsigned char *my_lds = lds + lane * RS;
    // 16 bytes of this lane's row into LDS at p (16-byte aligned when WIDE:
    // every lane's staging offset o_me is then a multiple of 16 bytes)
    auto stage16 = [](unsigned char *p, const uint4 &v) {
        if constexpr (WIDE) {
            *(uint4 *)p = v;
        } else {
            *(uint32_t *)(p) = v.x;
            *(uint32_t *)(p + 4) = v.y;
            *(uint32_t *)(p + 8) = v.z;
            *(uint32_t *)(p + 12) = v.w;
        }
    };
    // this lane's own row: offset past its first line and its last line (in
    // line units from the first)
    const uint32_t o_me = (uint32_t)((uintptr_t)(out0 + (uint64_t)lane * nb) & 127u);
    const uint64_t last_me = (o_me + nb - 1) / 128;
    // the rows this lane writes in store instruction j of a window
    const int chunk = lane % LPR;
    uint64_t rbase[NJ], rlast[NJ];
    uint32_t rflag[NJ];  // bit 0: row exists, 1: first line shared, 2: last line shared
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const uint64_t r = (uint64_t)(lane / LPR + RPI * j);
        const uintptr_t row = (uintptr_t)(out0 + r * nb);
        const uint32_t o = (uint32_t)(row & 127u);
        rbase[j] = (uint64_t)(row - o);
        rlast[j] = (o + nb - 1) / 128;
        rflag[j] = (r < nrows ? 1u : 0u) | (o ? 2u : 0u) | (((o + nb) & 127u) ? 4u : 0u);
    }
    // this row's first and last line, kept in registers
    uint4 f0, f1, f2, f3, f4, f5, f6, f7, l0, l1, l2, l3, l4, l5, l6, l7;
#define MRG_LOAD_LINE(x, p)                                                                  \
    do {                                                                                     \
        const unsigned char *p_ = (p);                                                      \
        x##0 = *(const uint4 *)(p_); x##1 = *(const uint4 *)(p_ + 16);                       \
        x##2 = *(const uint4 *)(p_ + 32); x##3 = *(const uint4 *)(p_ + 48);                  \
        x##4 = *(const uint4 *)(p_ + 64); x##5 = *(const uint4 *)(p_ + 80);                  \
        x##6 = *(const uint4 *)(p_ + 96); x##7 = *(const uint4 *)(p_ + 112);                 \
    } while (0)
#define MRG_STORE_LINE(x, p)                                                                 \
    do {                                                                                     \
        unsigned char *p_ = (p);                                                            \
        *(uint4 *)(p_) = x##0; *(uint4 *)(p_ + 16) = x##1;                                   \
        *(uint4 *)(p_ + 32) = x##2; *(uint4 *)(p_ + 48) = x##3;                              \
        *(uint4 *)(p_ + 64) = x##4; *(uint4 *)(p_ + 80) = x##5;                              \
        *(uint4 *)(p_ + 96) = x##6; *(uint4 *)(p_ + 112) = x##7;                             \
    } while (0)
    const uint64_t nsteps = (n + TV - 1) / TV;
    const uint64_t nwin = (nb + 127 + TB - 1) / TB;  // covers o + nb for any o < 128
    for (uint64_t k = 0; k < nwin; ++k) {
        if (k < nsteps) {
            const uint64_t cnt = n - k * TV < (uint64_t)TV ? n - k * TV : (uint64_t)TV;
            unsigned char *dst = my_lds + o_me;
            if (cnt == (uint64_t)TV) {
                if constexpr (G::kCheckedDraws) {
                    const G saved = g;
                    uint32_t neg = 0;
#pragma unroll
                    for (int q = 0; q < TB / 16; ++q) stage16(dst + q * 16, gen16<DT>(g, neg));
                    if (__any((int32_t)neg < 0)) {
                        g = saved;
#pragma unroll 1
                        for (int q = 0; q < TB / 16; ++q) {
                            stage16(dst + q * 16, gen16<DT>(g));
                        }
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < TB / 16; ++q) stage16(dst + q * 16, gen16<DT>(g));
                }
            } else {
                // the rows' last, shorter step (the same count in every lane)
                for (uint64_t c = 0; c < cnt; ++c) put1<DT>(dst + c * ES, g);
            }
        }
        __syncthreads();
        // keep this row's first line (window 0) and last line (its window)
        if (k == 0) MRG_LOAD_LINE(f, my_lds);
        if (last_me * 128 / TB == k) MRG_LOAD_LINE(l, my_lds + (last_me * 128 - k * TB));
        // the lines of window k that lie wholly in their row
        const uint64_t wof = k * TB + (uint64_t)chunk * 16;
        const uint64_t line = wof / 128;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const uint4 v = *(const uint4 *)(lds + (lane / LPR + RPI * j) * RS + chunk * 16);
            const bool whole = (rflag[j] & 1u) && line <= rlast[j] &&
                               !(line == 0 && (rflag[j] & 2u)) &&
                               !(line == rlast[j] && (rflag[j] & 4u));
            if (whole) *(uint4 *)(rbase[j] + wof) = v;
        }
        __syncthreads();
        // the spill past the window becomes the front of the next one
#pragma unroll
        for (int q = 0; q < 8; ++q) *(uint4 *)(my_lds + q * 16) = *(const uint4 *)(my_lds + TB + q * 16);
    }
    // shared lines: row r's first line holds row r-1's last bytes below o_r
    __syncthreads();
    MRG_STORE_LINE(f, my_lds);
    MRG_STORE_LINE(l, my_lds + 128);
#undef MRG_LOAD_LINE
#undef MRG_STORE_LINE
    __syncthreads();
    // 16 bytes per lane of each shared first line, 8 lanes per line, 8 rows
    // per step, four steps at a time: their LDS reads first, then the stores
    const int c16 = (lane & 7) * 16;
#pragma unroll 1
    for (int h = 0; h < 8; h += 4) {
        uint4 sv[4];
        uint32_t so[4];  // the row's o (0: nothing to write: first line whole, or no row)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint64_t r = (uint64_t)(8 * (h + j) + (lane >> 3));
            so[j] = r < nrows ? (uint32_t)((uintptr_t)(out0 + r * nb) & 127u) : 0u;
            // dword d: row r's own byte b >= o, else row r-1's last line (row
            // 0 reads its own window there and never writes those bytes)
            const uint32_t own = (uint32_t)r * RS, prev = r ? own - RS + 128 : own;
            uint32_t w[4];
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const uint32_t b = (uint32_t)c16 + 4 * d;
                w[d] = *(const uint32_t *)(lds + (b >= so[j] ? own : prev) + b);
            }
            sv[j] = make_uint4(w[0], w[1], w[2], w[3]);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (!so[j]) continue;
            const uint64_t r = (uint64_t)(8 * (h + j) + (lane >> 3));
            unsigned char *p = (unsigned char *)((uintptr_t)(out0 + r * nb) - so[j]) + c16;
            if (r > 0 || (uint32_t)c16 >= so[j]) {
                *(uint4 *)p = sv[j];
            } else {
                // the wave's first row: bytes below o belong to the previous wave
                const uint32_t w[4] = {sv[j].x, sv[j].y, sv[j].z, sv[j].w};
#pragma unroll
                for (int d = 0; d < 4; ++d)
                    if ((uint32_t)c16 + 4 * d >= so[j]) *(uint32_t *)(p + 4 * d) = w[d];
            }
        }
    }
    // the wave's last row ends in a line shared with the next wave's first:
    // its bytes there as dwords, one per lane
    {
        const uint64_t rl = nrows - 1;
        const uintptr_t row = (uintptr_t)(out0 + rl * nb);
        const uint32_t ol = (uint32_t)(row & 127u), el = (uint32_t)((ol + nb) & 127u);
        if ((uint32_t)lane * 4 < el) {
            unsigned char *p = (unsigned char *)(row - ol) + (ol + nb - 1) / 128 * 128;
            *(uint32_t *)(p + 4 * lane) = *(const uint32_t *)(lds + (uint32_t)rl * RS + 128 + 4 * lane);
        }
    }
}

// rows_fill_carry: rows_fill_carry_w with 16-byte staging when every row
// starts 16-byte aligned (the base and the row length), else dword staging.
template <int DT, int TB, class G>
__device__ __forceinline__ void rows_fill_carry(G &g, unsigned char *lds, int lane, uint64_t nrows,
                                                unsigned char *out0, uint64_t n)
{
    if ((uintptr_t)out0 % 16 == 0 && (n * Elem<DT>::size) % 16 == 0)
        rows_fill_carry_w<DT, TB, G, true>(g, lds, lane, nrows, out0, n);
    else
        rows_fill_carry_w<DT, TB, G, false>(g, lds, lane, nrows, out0, n);
}

// rows_fill_short: adjacent rows shorter than a line (n * ES < 128, row r at
// out0 + r * n * ES) are one block of nrows * n values.  Each lane stages its
// row in LDS (row r at r * n * ES, `lds` holding 64 * 128 bytes) and the wave
// copies the block out as dwords, 64 consecutive dwords per store.
template <int DT, class G>
__device__ __forceinline__ void rows_fill_short(G &g, unsigned char *lds, int lane,
                                                uint64_t nrows, unsigned char *out0, uint64_t n)
{
    constexpr int ES = Elem<DT>::size;
    if ((uint64_t)lane < nrows)
        for (uint64_t c = 0; c < n; ++c) put1<DT>(lds + (uint64_t)lane * n * ES + c * ES, g);
    __syncthreads();
    const uint64_t words = nrows * n * ES / 4;
    for (uint64_t i = lane; i < words; i += 64) ((uint32_t *)out0)[i] = ((const uint32_t *)lds)[i];
    __syncthreads();
}

// One 128-byte piece (128 / ES values) of a member's segment from g into
// LDS at pl.  With checked draws (GenF) the piece is drawn with the cheaper
// combination; when some lane's check fails the whole wave draws it again
// exactly, each lane from the state `at` values past w0 (the piece's first
// value: w0 is the chunk's first state).  g moves on by the piece either way.
template <int DT, class G>
__device__ __forceinline__ void draw_piece(G &g, unsigned char *pl, const uint32_t *w0, uint64_t at,
                                           const uint32_t *__restrict__ table)
{
    if constexpr (G::kCheckedDraws) {
        uint32_t neg = 0;
#pragma unroll
        for (int q = 0; q < 8; ++q) *(uint4 *)(pl + q * 16) = gen16<DT>(g, neg);
        if (__any((int32_t)neg < 0)) {
            uint32_t ps[6] = {w0[0], w0[1], w0[2], w0[3], w0[4], w0[5]};
            jump_global(table, at, 0, 0, 0, 16, ps);
            G ge;
            ge.load(ps);
#pragma unroll 1
            for (int q = 0; q < 8; ++q) *(uint4 *)(pl + q * 16) = gen16<DT>(ge);
        }
    } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) *(uint4 *)(pl + q * 16) = gen16<DT>(g);
    }
}

// ---------------------------------------------------------------------------
// wave_fill: values [v0, v1) of 64/GL streams at once, GL lanes per stream
// (lane l serves stream l / GL as its member g = l % GL).  Stream t of the
// wave is written at srow + t * row_stride + v * ES; only streams t < nsv
// are written.  Each lane's w holds its stream's state at v0 (the same in
// the GL lanes of a stream) and receives the state at v1 (want_end), else
// some state the caller must not use.
//
// Each stream first writes its head, the values before its row's first
// 128-byte line boundary (fewer than 128 / ES): value i of the head comes
// from A^i applied to the state (the head table of `tabs`: entry l is A^l),
// members taking i = g, GL + g, ..., and the stream moves on to the state
// A^head w.  The rest is cut into chunks of GL*L values; member g generates
// the L consecutive values [g*L, g*L + L) of each chunk starting from
// A^(g*L) applied to the chunk's first state (m: the lane's 18-word matrix
// pair), and the next chunk starts where member GL-1 ended (sequence
// splitting, sec. 2.3).  Every LDS flush of whole chunks writes aligned
// 128-byte lines.  In a chunk where rows end (and none goes on), members take
// only Lc <= L values each, the fewest whole pieces with GL*Lc covering the
// longest remaining row, starting from A^(g*Lc) (the Lc table of `tabs`); it
// writes the same lines up to each row's end (16-byte stores, dwords for the
// last group), and the stream's state is then moved over that chunk with the
// windowed tables.  `lds` holds 64 * 144 bytes.
// With a generator that has checked draws (GenF), each piece is drawn with
// the cheaper combination; in the rare piece where some lane's check fails,
// the whole wave draws the piece again exactly, from the chunk's first state
// jumped to the piece (the generator state itself is exact either way).
// NP: pieces each member stages per flush (1 or 2, dividing L / (128 / ES));
// with 2, every store instruction covers runs of two adjacent lines of one
// member instead of single lines 1 KiB apart (in a chunk where rows end the
// flush stays at one piece).  `lds` then holds 64 * (NP * 128 + 16) bytes.
// READ_ALL: read all LDS pieces of a flush before the first store (else each
// piece goes straight to memory).  AUX: cache policy of the whole-line stores.
// ---------------------------------------------------------------------------
template <int DT, int L, class G, bool READ_ALL = true, int GL = 64, int AUX = 0, int NP = 1>
__device__ __forceinline__ void wave_fill(uint32_t *w, const uint32_t *m, unsigned char *lds,
                                          int lane, unsigned char *srow, uint64_t row_stride,
                                          int nsv, uint64_t v0, uint64_t v1,
                                          const uint32_t *__restrict__ table,
                                          const uint32_t *__restrict__ tabs, bool want_end)
{
    constexpr int ES = Elem<DT>::size;
    constexpr int TV = 128 / ES;   // values per 128-byte piece
    constexpr int NH = L / TV;     // pieces per lane per chunk
    constexpr int RS = NP * 128 + 16;  // LDS row pitch (bytes)
    constexpr int SPW = 64 / GL;   // streams per wave
    constexpr int JPS = GL / 8;    // flush instructions per stream and piece
    constexpr int ROUNDS = (TV + GL - 1) / GL;  // head rounds (heads are < TV values)
    static_assert(NH >= 1 && L % TV == 0, "chunk must be whole pieces");
    static_assert((NP == 1 || NP == 2) && NH % NP == 0, "one or two pieces per flush");
    static_assert(GL == 64 || GL == 32 || GL == 16 || GL == 8, "8, 16, 32 or 64 lanes per stream");
    static_assert(ROUNDS * GL <= 64, "head table has 64 entries");
    const uint64_t chunk_vals = (uint64_t)GL * L;
    const uint64_t len = v1 > v0 ? v1 - v0 : 0;
    unsigned char *my_lds = lds + lane * RS;
    const int prow = lane >> 3;        // flush: 8 lanes per 128-byte piece
    const int pcol = (lane & 7) * 16;  //        8 pieces per instruction
    const int tl = lane / GL, gl = lane % GL;
    const int last = tl * GL + GL - 1;  // the member that ends a chunk

    // head of every stream (wave-uniform values, one per stream)
    uint32_t hvt[SPW];
#pragma unroll
    for (int t = 0; t < SPW; ++t)
        hvt[t] = (uint32_t)head_values<ES>(srow + t * row_stride + v0 * ES, len);
    uint32_t hv = hvt[0];
#pragma unroll
    for (int t = 1; t < SPW; ++t)
        if (tl == t) hv = hvt[t];
    if (__any(hv != 0u)) {
        uint32_t sel[6] = {w[0], w[1], w[2], w[3], w[4], w[5]};
        for (int k = 0; k < ROUNDS; ++k) {
            const uint32_t i = (uint32_t)(k * GL + gl);
            uint32_t hm[18];
#pragma unroll
            for (int q = 0; q < 18; ++q) hm[q] = tabs[(kHeadTable * 64 + i) * 18 + q];
            uint32_t st[6] = {w[0], w[1], w[2], w[3], w[4], w[5]};
            matvec3<C1>(hm, st[0], st[1], st[2]);
            matvec3<C2>(hm + 9, st[3], st[4], st[5]);
            if (tl < nsv && i < hv) {
                G g;
                g.load(st);
                put1<DT>(srow + tl * row_stride + (v0 + i) * ES, g);
            }
            if (i == hv) {
#pragma unroll
                for (int q = 0; q < 6; ++q) sel[q] = st[q];
            }
        }
        // the state at v0 + hv sits with member hv % GL of this stream
#pragma unroll
        for (int q = 0; q < 6; ++q) w[q] = __shfl(sel[q], tl * GL + (int)(hv % GL));
    }
    const uint64_t start = v0 + hv;  // this lane's stream: first line-aligned value

    bool whole = true;
    for (uint64_t c = 0;; ++c) {
        const uint64_t c0 = start + c * chunk_vals;
        if (!__any(c0 < v1)) break;
        const bool active = c0 < v1;
        const bool full = c0 + chunk_vals <= v1;
        const bool cut = __any(tl < nsv && active && !full);  // a row ends in this chunk
        // members' values this chunk: L, or in a chunk where every row ends,
        // the fewest whole pieces that cover the longest of them
        uint32_t Lc = L;
        if (cut) {
            uint64_t rmax = 0;
#pragma unroll
            for (int t = 0; t < SPW; ++t) {
                const uint64_t ct = v0 + hvt[t] + c * chunk_vals;
                const uint64_t r = (SPW > 1 && t >= nsv) || ct >= v1 ? 0 : v1 - ct;
                rmax = r > rmax ? r : rmax;
            }
            if (rmax < chunk_vals) {
                const uint64_t per = (rmax + GL - 1) / GL;
                Lc = (uint32_t)((per + TV - 1) / TV * TV);
            }
        }
        const int h_end = (int)(Lc / TV);
        uint32_t st[6] = {w[0], w[1], w[2], w[3], w[4], w[5]};
        if (Lc == (uint32_t)L) {
            matvec3<C1>(m, st[0], st[1], st[2]);
            matvec3<C2>(m + 9, st[3], st[4], st[5]);
        } else {
            const uint32_t *mc = tabs + ((uint32_t)lane_table((int)Lc) * 64 + gl) * 18;
            matvec3<C1>(mc, st[0], st[1], st[2]);
            matvec3<C2>(mc + 9, st[3], st[4], st[5]);
        }
        G g;
        g.load(st);
        // piece h + p of this member (gl*Lc + (h+p)*TV values into the
        // chunk) into its LDS row at p * 128
        auto draw = [&](int h, int p) {
            draw_piece<DT>(g, my_lds + p * 128, w, (uint64_t)gl * Lc + (uint64_t)(h + p) * TV,
                           table);
        };
        if (!cut) {
            // whole chunks: NP pieces per member per flush; store instruction
            // j takes the NP-piece runs of the 8 / NP lanes (members) 8j / NP
            // ...: lane group prow writes piece P = 8j + prow, i.e. piece
            // h + P % NP of lane P / NP, an aligned 128-byte line of that
            // member's row; all lanes of one instruction serve one stream
            constexpr int NJ = 8 * NP;
            // per stream of the wave: written in this chunk or not, and a
            // descriptor based at its chunk (the pieces then differ only by
            // the per-lane offset and the flush's uniform offset)
            __amdgpu_buffer_rsrc_t rs[SPW];
            uint32_t live = 0;
#pragma unroll
            for (int t = 0; t < SPW; ++t) {
                const uint64_t ct = v0 + hvt[t] + c * chunk_vals;
                if (!((SPW > 1 && t >= nsv) || ct + chunk_vals > v1)) live |= 1u << t;
                rs[t] = uniform_rsrc(srow + t * row_stride + ct * ES, (uint32_t)(GL * L * ES));
            }
            for (int h = 0; h < NH; h += NP) {
#pragma unroll
                for (int p = 0; p < NP; ++p) draw(h, p);
                __syncthreads();
                if constexpr (READ_ALL) {
                    uint4 v[NJ];
#pragma unroll
                    for (int j = 0; j < NJ; ++j) {
                        const int P = 8 * j + prow;
                        v[j] = *(const uint4 *)(lds + (P / NP) * RS + (P % NP) * 128 + pcol);
                    }
#pragma unroll
                    for (int j = 0; j < NJ; ++j) {
                        const int t = j / (JPS * NP);
                        if (!((live >> t) & 1u)) continue;
                        const int P = 8 * j + prow;
                        const uint32_t loff =
                            (uint32_t)(((P / NP) % GL) * L * ES + (P % NP) * 128 + pcol);
                        store16_rsrc<AUX>(rs[t], loff, (uint32_t)(h * TV * ES), v[j]);
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < NJ; ++j) {
                        const int t = j / (JPS * NP);
                        if (!((live >> t) & 1u)) continue;
                        const int P = 8 * j + prow;
                        const uint4 v =
                            *(const uint4 *)(lds + (P / NP) * RS + (P % NP) * 128 + pcol);
                        const uint32_t loff =
                            (uint32_t)(((P / NP) % GL) * L * ES + (P % NP) * 128 + pcol);
                        store16_rsrc<AUX>(rs[t], loff, (uint32_t)(h * TV * ES), v);
                    }
                }
                __syncthreads();
            }
        } else {
            // some row ends here: one piece per flush, 16-byte stores below
            // the end and dword stores for the group that straddles it
            for (int h = 0; h < h_end; ++h) {
                draw(h, 0);
                __syncthreads();
                // piece row prow + 8j is stream j / JPS, member prow + 8 (j % JPS)
#pragma unroll 1
                for (int j = 0; j < 8; ++j) {
                    const int t = j / JPS;
                    if (SPW > 1 && t >= nsv) break;
                    // stream t's head count sits in its first lane
                    const uint32_t ht = (uint32_t)__builtin_amdgcn_readlane((int)hv, t * GL);
                    const uint64_t ct = v0 + ht + c * chunk_vals;
                    if (ct >= v1) continue;
                    const uint64_t rem = (v1 - ct < chunk_vals ? v1 - ct : chunk_vals) * ES;
                    const uint32_t o = (uint32_t)((prow + 8 * (j % JPS)) * Lc * ES + pcol + h * 128);
                    if (o >= rem) continue;
                    const uint4 v = *(const uint4 *)(lds + (prow + 8 * j) * RS + pcol);
                    unsigned char *p = srow + t * row_stride + ct * ES + o;
                    if (o + 16 <= rem) {
                        *(uint4 *)p = v;
                    } else {
                        *(uint32_t *)p = v.x;
                        if (o + 4 < rem) *(uint32_t *)(p + 4) = v.y;
                        if (o + 8 < rem) *(uint32_t *)(p + 8) = v.z;
                    }
                }
                __syncthreads();
            }
        }
        if (full) {  // member GL-1 ends at the next chunk's first state
            uint32_t e[6];
            g.store(e);
#pragma unroll
            for (int k = 0; k < 6; ++k) w[k] = __shfl(e[k], last);
        } else if (active) {
            whole = false;
        }
    }
    // w is the last chunk's first state: move it over the partial chunk
    if (!whole && want_end) jump_global(table, (v1 - start) % chunk_vals, 0, 0, 0, 16, w);
}

// ---------------------------------------------------------------------------
// wave_fill_whole: wave_fill(w, ..., 0, n, ..., want_end) for the bulk case
// where every chunk is whole and every row starts on a line: 64/GL full
// streams of n values, n a multiple of the chunk GL*L, srow 128-byte aligned,
// row pitch n*ES a multiple of 128, and the group's 64/GL rows addressable
// from srow with 32-bit offsets (64/GL * n * ES < 2^32).  One descriptor for
// the group; a store's lane offset is fixed by its piece slot and the flush
// adds a wave-uniform offset.  Same outputs and end states as wave_fill.
// ---------------------------------------------------------------------------
template <int DT, int L, class G, int GL, int NP, int AUX = 0>
__device__ __forceinline__ void wave_fill_whole(uint32_t *w, const uint32_t *m, unsigned char *lds,
                                                int lane, unsigned char *srow, uint64_t n,
                                                const uint32_t *__restrict__ table)
{
    constexpr int ES = Elem<DT>::size;
    constexpr int TV = 128 / ES;       // values per 128-byte piece
    constexpr int NH = L / TV;         // pieces per lane per chunk
    constexpr int RS = NP * 128 + 16;  // LDS row pitch (bytes)
    constexpr int SPW = 64 / GL;
    constexpr int NJ = 8 * NP;         // store instructions per flush
    static_assert((NP == 1 || NP == 2) && NH % NP == 0, "one or two pieces per flush");
    const int tl = lane / GL, gl = lane % GL;
    const int prow = lane >> 3, pcol = (lane & 7) * 16;
    unsigned char *my_lds = lds + lane * RS;
    const uint32_t row_bytes = (uint32_t)(n * ES);
    const __amdgpu_buffer_rsrc_t rsrc = uniform_rsrc(srow, SPW * row_bytes);
    const uint64_t nchunks = n / ((uint64_t)GL * L);
    for (uint64_t c = 0; c < nchunks; ++c) {
        uint32_t st[6] = {w[0], w[1], w[2], w[3], w[4], w[5]};
        matvec3<C1>(m, st[0], st[1], st[2]);
        matvec3<C2>(m + 9, st[3], st[4], st[5]);
        G g;
        g.load(st);
        for (int h = 0; h < NH; h += NP) {
#pragma unroll
            for (int p = 0; p < NP; ++p)
                draw_piece<DT>(g, my_lds + p * 128, w, (uint64_t)gl * L + (uint64_t)(h + p) * TV,
                               table);
            __syncthreads();
            // store j: piece P = 8j + prow is piece h + P % NP of lane P / NP
            uint4 v[NJ];
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const int P = 8 * j + prow;
                v[j] = *(const uint4 *)(lds + (P / NP) * RS + (P % NP) * 128 + pcol);
            }
            const uint32_t soff = (uint32_t)((c * GL * L + (uint64_t)h * TV) * ES);
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const int P = 8 * j + prow, owner = P / NP;
                const uint32_t voff = (uint32_t)(owner / GL) * row_bytes +
                                      (uint32_t)((owner % GL) * L * ES + (P % NP) * 128 + pcol);
                store16_rsrc<AUX>(rsrc, voff, soff, v[j]);
            }
            __syncthreads();
        }
        // member GL-1 ends at the next chunk's first state
        uint32_t e[6];
        g.store(e);
#pragma unroll
        for (int k = 0; k < 6; ++k) w[k] = __shfl(e[k], tl * GL + GL - 1);
    }
}

// Workgroups are dispatched to the 8 XCDs in turn (workgroup b on XCD b % 8).
// xcd_range gives the workgroups of each XCD a contiguous range of the items,
// so that work which varies with the item index in a period dividing 8 still
// spreads evenly over the XCDs, and neighbouring rows meet in one L2.
struct XcdRange { uint64_t first, end, step; };
__device__ __forceinline__ XcdRange xcd_range(uint64_t items)
{
    const uint64_t nb = gridDim.x, b = blockIdx.x;
    if (nb < 8) return {b, items, nb};
    const uint64_t x = b % 8, q = items / 8, r = items % 8;
    const uint64_t lo = x * q + (x < r ? x : r);
    return {lo + b / 8, lo + q + (x < r ? 1 : 0), (nb - x + 7) / 8};
}

// The chunked order, for one workgroup per item: in each super-chunk of 8*Q
// items, XCD x takes the Q consecutive items [x*Q, x*Q + Q) (its workgroups
// in dispatch order), so each XCD works on contiguous runs while all XCDs move
// through memory together, one front of writes instead of eight.  Items past
// the last whole super-chunk keep their own index.
__device__ __forceinline__ XcdRange xcd_chunk(uint64_t items)
{
    constexpr uint64_t Q = 64, S = 8 * Q;
    const uint64_t b = blockIdx.x;
    if (gridDim.x != items || b >= items / S * S) return {b, b + 1, 1};
    const uint64_t l = b % S;
    const uint64_t g = b - l + (l % 8) * Q + l / 8;
    return {g, g + 1, 1};
}

}  // namespace mrg
