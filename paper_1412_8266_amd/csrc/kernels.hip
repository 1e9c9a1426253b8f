// HIP kernels of the MRG32k3a stream library (gfx950, wave64).
//
//   init_kernel      stream-set creation: state_g = A^(g * 2^127) seed     (sec. 4.1, 5.1)
//   jump_kernel      per-stream jump ahead with 4-bit windowed tables of
//                    A^(d * 16^w) mod m staged in LDS                    (sec. 2.3)
//   jumpu_kernel     one jump matrix (formed on the host) for every stream
//   fill_sm_kernel   bulk generation, stream-major output, one stream per
//                    lane, state in registers, LDS transpose to 16-byte
//                    row-segment stores                                  (sec. 5.2, Listing 1)
//   fill_il_kernel   bulk generation, interleaved output (lane = stream,
//                    consecutive lanes write consecutive elements)
//   fill_coop_kernel bulk generation, stream-major output, GL lanes per
//                    stream (sequence splitting inside each stream)
//   random_init_kernel  random spacing: each stream from its own expanded
//                    SplitMix64 draw                                     (sec. 2.3)
//   fill_split_kernel   one stream's outputs in order, split into blocks
//   fill_leap_kernel    leapfrog: one stream dealt to P players, each
//                    player's cards in a row                            (sec. 2.3)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gen_device.hpp"
#include "kernels.h"

namespace mrg {

// Stage windows [w_lo, w_hi) of both components into LDS, then apply them.
__global__ void __launch_bounds__(256)
jump_kernel(uint32_t *__restrict__ planes, uint64_t plane_stride, uint64_t first,
            uint64_t count, const uint64_t *__restrict__ exps, uint64_t g0,
            InitSeed seed, const uint32_t *__restrict__ table, int w_lo, int w_hi)
{
    extern __shared__ uint32_t tab[];
    const int nw = (w_hi - w_lo) * kTableWindowWords;  // words per component
    for (int i = threadIdx.x; i < nw; i += blockDim.x) {
        tab[i] = table[(0 * kTableWindows + w_lo) * kTableWindowWords + i];
        tab[nw + i] = table[(1 * kTableWindows + w_lo) * kTableWindowWords + i];
    }
    __syncthreads();

    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = s < count;
    uint32_t a0 = 0, a1 = 0, a2 = 0, b0 = 0, b1 = 0, b2 = 0;
    uint64_t e0 = 0, e1 = 0, e2 = 0;
    const uint64_t idx = first + s;
    if (active) {
        if (exps) {  // jump the current state by its own exponent
            a0 = planes[0 * plane_stride + idx];
            a1 = planes[1 * plane_stride + idx];
            a2 = planes[2 * plane_stride + idx];
            b0 = planes[3 * plane_stride + idx];
            b1 = planes[4 * plane_stride + idx];
            b2 = planes[5 * plane_stride + idx];
            e0 = exps[3 * s + 0];
            e1 = exps[3 * s + 1];
            e2 = exps[3 * s + 2];
        } else {     // create: start of global stream g = g0 + s is A^(g 2^127) seed
            a0 = seed.w[0]; a1 = seed.w[1]; a2 = seed.w[2];
            b0 = seed.w[3]; b1 = seed.w[4]; b2 = seed.w[5];
            const uint64_t g = g0 + s;
            e0 = 0;
            e1 = (g & 1u) << 63;
            e2 = g >> 1;
        }
    }
    for (int w = w_lo; w < w_hi; ++w) {
        const uint32_t d = exp_digit(e0, e1, e2, w);
        if (!__any(d != 0u)) continue;  // wave-uniform skip of empty windows
        const uint32_t *T1 = tab + ((w - w_lo) * 16 + d) * 9;
        const uint32_t *T2 = tab + nw + ((w - w_lo) * 16 + d) * 9;
        matvec3<C1>(T1, a0, a1, a2);
        matvec3<C2>(T2, b0, b1, b2);
    }
    if (active) {
        planes[0 * plane_stride + idx] = canon1(a0);
        planes[1 * plane_stride + idx] = canon1(a1);
        planes[2 * plane_stride + idx] = canon1(a2);
        planes[3 * plane_stride + idx] = canon2(b0);
        planes[4 * plane_stride + idx] = canon2(b1);
        planes[5 * plane_stride + idx] = canon2(b2);
    }
}

__global__ void __launch_bounds__(256)
jumpu_kernel(uint32_t *__restrict__ planes, uint64_t plane_stride, uint64_t first,
             uint64_t count, JumpMatrices J)
{
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= count) return;
    const uint64_t idx = first + s;
    uint32_t a0 = planes[0 * plane_stride + idx];
    uint32_t a1 = planes[1 * plane_stride + idx];
    uint32_t a2 = planes[2 * plane_stride + idx];
    uint32_t b0 = planes[3 * plane_stride + idx];
    uint32_t b1 = planes[4 * plane_stride + idx];
    uint32_t b2 = planes[5 * plane_stride + idx];
    matvec3<C1>(J.m, a0, a1, a2);
    matvec3<C2>(J.m + 9, b0, b1, b2);
    planes[0 * plane_stride + idx] = a0;
    planes[1 * plane_stride + idx] = a1;
    planes[2 * plane_stride + idx] = a2;
    planes[3 * plane_stride + idx] = b0;
    planes[4 * plane_stride + idx] = b1;
    planes[5 * plane_stride + idx] = b2;
}

// Random spacing (sec. 2.3): stream g = g0 + s starts at the state expanded
// from SplitMix64 output g of the master seed.
__global__ void __launch_bounds__(256)
random_init_kernel(uint32_t *__restrict__ planes, uint64_t plane_stride, uint64_t count,
                   uint64_t g0, uint64_t master)
{
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= count) return;
    uint32_t w[6];
    expand_seed(splitmix64_mix(master + (g0 + s + 1) * kSplitMixGamma), w);
    store_state(planes, plane_stride, s, w);
}

// ---------------------------------------------------------------------------
// generation
// ---------------------------------------------------------------------------
// Lane-per-stream stream-major fill: one wave per 64 streams, each lane
// generating its stream's n values through the LDS tile writer rows_fill.
template <int DT, int TB, class G>
__global__ void __launch_bounds__(64)
fill_sm_kernel(uint32_t *__restrict__ planes, uint64_t plane_stride, uint64_t first,
               uint64_t count, uint64_t n, unsigned char *__restrict__ out)
{
    constexpr int ES = Elem<DT>::size;
    // TB = 0: rows off their lines, written by rows_fill_carry in 128-byte windows
    __shared__ __attribute__((aligned(16))) unsigned char lds[64 * (TB ? TB + 16 : 128 + 160)];
    const int lane = threadIdx.x;
    const uint64_t s0 = (uint64_t)blockIdx.x * 64;
    const uint64_t nrows = count - s0 < 64 ? count - s0 : 64;
    const bool active = (uint64_t)lane < nrows;
    const uint64_t idx = first + s0 + lane;

    uint32_t w[6] = {1u, 1u, 1u, 1u, 1u, 1u};
    if (active) load_state(planes, plane_stride, idx, w);
    G g;
    g.load(w);
    if (n * ES < 128) {  // the wave's rows are one block shorter than 64 lines
        rows_fill_short<DT, G>(g, lds, lane, nrows, out + s0 * n * ES, n);
    } else {
        if constexpr (TB == 0)
            rows_fill_carry<DT, 128, G>(g, lds, lane, nrows, out + s0 * n * ES, n);
        else
            rows_fill<DT, TB, G>(g, lds, lane, nrows, out + s0 * n * ES, n * ES, n);
    }
    if (active) {
        g.store(w);
        store_state(planes, plane_stride, idx, w);
    }
}

// Interleaved output out[k * count + s]: consecutive lanes are consecutive
// streams, so each step is one coalesced store per wave.  Written with the
// per-thread stream object of the public device header, as a user kernel
// would draw: one stream per thread, next() per value.
template <int DT, class G>
__global__ void __launch_bounds__(256)
fill_il_kernel(uint32_t *__restrict__ planes, uint64_t plane_stride, uint64_t first,
               uint64_t count, uint64_t n, unsigned char *__restrict__ out)
{
    constexpr int ES = Elem<DT>::size;
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= count) return;
    Stream<G> rng;
    rng.load(planes, plane_stride, first + s);
    unsigned char *p = out + s * ES;
    const uint64_t step = count * ES;
    uint64_t k = 0;
    for (; k + 4 <= n; k += 4) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            put1<DT>(p, rng.g);
            p += step;
        }
    }
    for (; k < n; ++k) {
        put1<DT>(p, rng.g);
        p += step;
    }
    rng.store(planes, plane_stride, first + s);
}

// Wave-per-stream stream-major fill: workgroups (one wave each) stride over
// groups of 64/GL streams, GL lanes per stream; each group is written by
// wave_fill, so that every flush writes whole 128-byte lines and the streams
// in flight stay adjacent.  Lanes of a group past the last stream run on a
// dummy state and write nothing.  Groups go to XCDs by xcd_chunk (or
// xcd_range), gen_device.hpp.  Members stage two pieces per flush when their
// chunk segment holds an even number of them (runs of two lines per member
// per store instruction: 4 % faster on 2^20 x 4096 uint32 than one piece, at
// 17 KiB of LDS per wave, two waves per SIMD); else one (9 KiB, four waves
// per SIMD).  The bound keeps the register count inside that occupancy.
template <int DT, int L>
constexpr int coop_pieces() { return (L / (128 / Elem<DT>::size)) % 2 == 0 ? 2 : 1; }

template <int DT, int L, int GL, class G>
__global__ void __launch_bounds__(64, (coop_pieces<DT, L>() == 2 ? 2 : 4))
fill_coop_kernel(uint32_t *__restrict__ planes, uint64_t plane_stride, uint64_t first,
                 uint64_t count, uint64_t n, unsigned char *__restrict__ out,
                 const uint32_t *__restrict__ lane_tab, const uint32_t *__restrict__ tabs,
                 const uint32_t *__restrict__ table, int order, int whole)
{
    constexpr int ES = Elem<DT>::size;
    constexpr int SPW = 64 / GL;
    constexpr int NP = coop_pieces<DT, L>();
    __shared__ __attribute__((aligned(16))) unsigned char lds[64 * (NP * 128 + 16)];
    const int lane = threadIdx.x;
    const int t = lane / GL;  // this lane's stream within the group

    const uint64_t groups = (count + SPW - 1) / SPW;
    const XcdRange R = order == 0 && gridDim.x == groups ? xcd_chunk(groups) : xcd_range(groups);
    for (uint64_t grp = R.first; grp < R.end; grp += R.step) {
        const uint64_t s0 = grp * SPW;
        const int nsv = count - s0 < (uint64_t)SPW ? (int)(count - s0) : SPW;
        const uint64_t idx = first + s0 + t;
        uint32_t w[6] = {1u, 1u, 1u, 1u, 1u, 1u};
        if (t < nsv) load_state(planes, plane_stride, idx, w);
        // this member's lane matrix, loaded per group (L2-resident) so that it
        // holds no registers while the group's values are drawn
        uint32_t m[18];
#pragma unroll
        for (int i = 0; i < 18; ++i) m[i] = lane_tab[(lane % GL) * 18 + i];
        if (whole && nsv == SPW)  // every chunk whole, rows on lines (checked on the host)
            wave_fill_whole<DT, L, G, GL, NP>(w, m, lds, lane, out + s0 * n * ES, n, table);
        else
            wave_fill<DT, L, G, true, GL, 0, NP>(w, m, lds, lane, out + s0 * n * ES, n * ES, nsv, 0,
                                                 n, table, tabs, true);
        if (lane % GL == 0 && t < nsv) store_state(planes, plane_stride, idx, w);
    }
}

// Sequence splitting of one stream (sec. 2.3): its outputs [0, N) in order as
// blocks of B values (the last one rem values when rem > 0), block r starting
// from A^(r*B) applied to the stream state (stream sidx of the planes) and
// written by one wave with wave_fill (64 lanes, L values per lane per chunk).
// Each XCD takes one contiguous range of blocks (measured 4 % faster here than
// the chunked order of the stream-major fill).  The stream state is not
// advanced here.
template <int DT, int L, class G>
__global__ void __launch_bounds__(64)
fill_split_kernel(const uint32_t *__restrict__ planes, uint64_t plane_stride, uint64_t sidx,
                  uint64_t nfull, uint64_t B, uint64_t rem, unsigned char *__restrict__ out,
                  const uint32_t *__restrict__ lane_tab, const uint32_t *__restrict__ tabs,
                  const uint32_t *__restrict__ table)
{
    constexpr int ES = Elem<DT>::size;
    __shared__ __attribute__((aligned(16))) unsigned char lds[64 * 144];
    const int lane = threadIdx.x;
    uint32_t m[18];
#pragma unroll
    for (int i = 0; i < 18; ++i) m[i] = lane_tab[lane * 18 + i];
    uint32_t s0[6];
    load_state(planes, plane_stride, sidx, s0);
    const XcdRange R = xcd_range(nfull + (rem ? 1 : 0));
    for (uint64_t r = R.first; r < R.end; r += R.step) {
        uint32_t w[6] = {s0[0], s0[1], s0[2], s0[3], s0[4], s0[5]};
        jump_global(table, r * B, 0, 0, 0, 16, w);
        wave_fill<DT, L, G, true, 64>(w, m, lds, lane, out + r * B * ES, B * ES, 1, 0,
                                      r < nfull ? B : rem, table, tabs, false);
    }
}

// Leapfrog (sec. 2.3) with each player's cards in a row: card k of player t
// is output t + k*P of the stream (stream sidx of the planes) and goes to
// out[t*K + k].  A column block is KB = min(K, 64) card columns; lane
// l < R*KB (R = 64 / KB) takes column k = KB*kb + l % KB and sub-segment
// r = l / KB of each segment of T = R*Ts players, i.e. the stream's outputs
// [k*P + t0 + r*Ts, ... + Ts) in order, written down its column: a store
// instruction covers R runs of KB adjacent cards (64 adjacent cards when
// K >= 64).  Work items are (column block kb, segment); each workgroup takes
// a contiguous run of the nkb * nseg items, jumps its lanes once (A^(k*P +
// t0 + r*Ts)) and from then on only continues: to the next segment by
// A^(T - Ts) (Jseg; stepping on when R = 1), to the next column block by
// A^(63*P) (J63; only with R = 1, since K < 64 leaves one column block).  The
// stream state is not advanced here.
template <int DT, class G>
__global__ void __launch_bounds__(64)
fill_leap_kernel(const uint32_t *__restrict__ planes, uint64_t plane_stride, uint64_t sidx,
                 LeapArgs A, unsigned char *__restrict__ out, const uint32_t *__restrict__ table)
{
    constexpr int ES = Elem<DT>::size;
    const uint64_t lane = threadIdx.x;
    const uint64_t nb = gridDim.x, b = blockIdx.x;
    const uint64_t q = A.items / nb, rr = A.items % nb;
    const uint64_t i0 = b * q + (b < rr ? b : rr);
    const uint64_t i1 = i0 + q + (b < rr ? 1 : 0);
    if (i0 >= i1 || lane >= (uint64_t)A.R * A.KB) return;
    const uint64_t kl = lane % A.KB, r = lane / A.KB;
    uint64_t kb = i0 / A.nseg, seg = i0 % A.nseg;
    uint32_t w[6];
    load_state(planes, plane_stride, sidx, w);
    {
        // lanes past the last column start anywhere in range and write nothing
        const uint64_t k = kb * A.KB + kl < A.K ? kb * A.KB + kl : A.K - 1;
        const uint64_t t = seg * A.T + r * A.Ts < A.P ? seg * A.T + r * A.Ts : A.P - 1;
        jump_global(table, k * A.P + t, 0, 0, 0, 16, w);
    }
    G g;
    g.load(w);
    const uint64_t row = A.K * ES;
    for (uint64_t it = i0; it < i1; ++it) {
        if (it != i0) {
            if (seg == 0) {
                // column k ended at output (k+1)*P; column k+64 starts at (k+64)*P
                g.store(w);
                matvec3<C1>(A.J63.m, w[0], w[1], w[2]);
                matvec3<C2>(A.J63.m + 9, w[3], w[4], w[5]);
                g.load(w);
            } else if (A.R > 1) {
                // sub-segment r ended at t0 + (r+1)*Ts; the next one starts T - Ts on
                g.store(w);
                matvec3<C1>(A.Jseg.m, w[0], w[1], w[2]);
                matvec3<C2>(A.Jseg.m + 9, w[3], w[4], w[5]);
                g.load(w);
            }
        }
        const uint64_t k = kb * A.KB + kl;
        const uint64_t t0 = seg * A.T + r * A.Ts;
        const uint64_t t1 = t0 + A.Ts < A.P ? t0 + A.Ts : A.P;
        if (k < A.K && t0 < t1) {
            unsigned char *p = out + (t0 * A.K + k) * ES;
            uint64_t t = t0;
            for (; t + 4 <= t1; t += 4) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    put1<DT>(p, g);
                    p += row;
                }
            }
            for (; t < t1; ++t) {
                put1<DT>(p, g);
                p += row;
            }
        }
        if (++seg == A.nseg) {
            seg = 0;
            ++kb;
        }
    }
}

// ---------------------------------------------------------------------------
// launchers (host side)
// ---------------------------------------------------------------------------
static unsigned grid_of(uint64_t items, unsigned block)
{
    return (unsigned)((items + block - 1) / block);
}

hipError_t launch_init(uint32_t *planes, uint64_t plane_stride, uint64_t count,
                       uint64_t g0, const InitSeed &seed, const uint32_t *table,
                       int w_lo, int w_hi, hipStream_t st)
{
    const size_t lds = (size_t)2 * (w_hi - w_lo) * kTableWindowWords * sizeof(uint32_t);
    hipLaunchKernelGGL(jump_kernel, dim3(grid_of(count, 256)), dim3(256), lds, st, planes,
                       plane_stride, (uint64_t)0, count, (const uint64_t *)nullptr, g0, seed,
                       table, w_lo, w_hi);
    return hipGetLastError();
}

hipError_t launch_jump(uint32_t *planes, uint64_t plane_stride, uint64_t first,
                       uint64_t count, const uint64_t *d_exp, const uint32_t *table,
                       hipStream_t st)
{
    const int w_lo = 0, w_hi = kTableWindows;
    const size_t lds = (size_t)2 * (w_hi - w_lo) * kTableWindowWords * sizeof(uint32_t);
    InitSeed none = {};
    hipLaunchKernelGGL(jump_kernel, dim3(grid_of(count, 256)), dim3(256), lds, st, planes,
                       plane_stride, first, count, d_exp, (uint64_t)0, none, table, w_lo, w_hi);
    return hipGetLastError();
}

hipError_t launch_jump_uniform(uint32_t *planes, uint64_t plane_stride, uint64_t first,
                               uint64_t count, const JumpMatrices &J, hipStream_t st)
{
    hipLaunchKernelGGL(jumpu_kernel, dim3(grid_of(count, 256)), dim3(256), 0, st, planes,
                       plane_stride, first, count, J);
    return hipGetLastError();
}

template <int DT, class G>
static hipError_t launch_fill_g(uint32_t *planes, uint64_t plane_stride, uint64_t first,
                                uint64_t count, uint64_t n, int layout, void *out,
                                const FillLaunch &fl, int tile_bytes, hipStream_t st)
{
    unsigned char *o = (unsigned char *)out;
    if (layout == 1) {
        hipLaunchKernelGGL((fill_il_kernel<DT, G>), dim3(grid_of(count, 256)), dim3(256), 0, st,
                           planes, plane_stride, first, count, n, o);
    } else if (fl.kernel == 1) {
        constexpr int TV = 128 / Elem<DT>::size;  // values per 128-byte piece
        const dim3 grid(fl.grid), block(64);
        const int nh = fl.L / TV;
#define MRG_COOP(GL, NH)                                                                        \
    hipLaunchKernelGGL((fill_coop_kernel<DT, (NH) * TV, GL, G>), grid, block, 0, st, planes,     \
                       plane_stride, first, count, n, o, fl.lane_tab, fl.tabs, fl.table,   \
                       fl.order, fl.whole)
        if (fl.L % TV) return hipErrorInvalidValue;
        else if (fl.lanes == 64 && nh == 1) MRG_COOP(64, 1);
        else if (fl.lanes == 64 && nh == 2) MRG_COOP(64, 2);
        else if (fl.lanes == 32 && nh == 2) MRG_COOP(32, 2);
        else if (fl.lanes == 32 && nh == 4) MRG_COOP(32, 4);
        else if (fl.lanes == 16 && nh == 4) MRG_COOP(16, 4);
        else if (fl.lanes == 16 && nh == 8) MRG_COOP(16, 8);
        else if (fl.lanes == 8 && nh == 8) MRG_COOP(8, 8);
        else if (fl.lanes == 8 && nh == 16) MRG_COOP(8, 16);
        else return hipErrorInvalidValue;
#undef MRG_COOP
    } else if (tile_bytes == 0 && ((uintptr_t)out % 128 || (n * Elem<DT>::size) % 128)) {
        // rows off their lines: one write per shared line (rows_fill_carry)
        hipLaunchKernelGGL((fill_sm_kernel<DT, 0, G>), dim3(grid_of(count, 64)), dim3(64), 0, st,
                           planes, plane_stride, first, count, n, o);
    } else if (tile_bytes == 256 || (tile_bytes == 0 && n * Elem<DT>::size >= 1024)) {
        hipLaunchKernelGGL((fill_sm_kernel<DT, 256, G>), dim3(grid_of(count, 64)), dim3(64), 0, st,
                           planes, plane_stride, first, count, n, o);
    } else {
        hipLaunchKernelGGL((fill_sm_kernel<DT, 128, G>), dim3(grid_of(count, 64)), dim3(64), 0, st,
                           planes, plane_stride, first, count, n, o);
    }
    return hipGetLastError();
}

template <class G>
static hipError_t launch_fill_d(uint32_t *planes, uint64_t plane_stride, uint64_t first,
                                uint64_t count, uint64_t n, int dtype, int layout, void *out,
                                const FillLaunch &fl, int tile_bytes, hipStream_t st)
{
    switch (dtype) {
    case 0: return launch_fill_g<0, G>(planes, plane_stride, first, count, n, layout, out, fl, tile_bytes, st);
    case 1: return launch_fill_g<1, G>(planes, plane_stride, first, count, n, layout, out, fl, tile_bytes, st);
    default: return launch_fill_g<2, G>(planes, plane_stride, first, count, n, layout, out, fl, tile_bytes, st);
    }
}

hipError_t launch_fill(uint32_t *planes, uint64_t plane_stride, uint64_t first, uint64_t count,
                       uint64_t n, int dtype, int layout, void *out,
                       const FillLaunch &fl, const FillTuning &tune, hipStream_t st)
{
    if (tune.engine == 1)
        return launch_fill_d<GenF>(planes, plane_stride, first, count, n, dtype, layout, out, fl,
                                   tune.tile_bytes, st);
    return launch_fill_d<GenI>(planes, plane_stride, first, count, n, dtype, layout, out, fl,
                               tune.tile_bytes, st);
}

hipError_t launch_random_init(uint32_t *planes, uint64_t plane_stride, uint64_t count,
                              uint64_t g0, uint64_t master, hipStream_t st)
{
    hipLaunchKernelGGL(random_init_kernel, dim3(grid_of(count, 256)), dim3(256), 0, st, planes,
                       plane_stride, count, g0, master);
    return hipGetLastError();
}

template <int DT, class G>
static hipError_t launch_partition_g(const uint32_t *planes, uint64_t plane_stride, uint64_t sidx,
                                     const PartitionLaunch &pl, void *out, hipStream_t st)
{
    unsigned char *o = (unsigned char *)out;
    constexpr int TV = 128 / Elem<DT>::size;
    if (pl.kind == 0) {
        if (pl.L == TV)
            hipLaunchKernelGGL((fill_split_kernel<DT, TV, G>), dim3(pl.grid), dim3(64), 0, st, planes,
                               plane_stride, sidx, pl.nfull, pl.B, pl.rem, o, pl.lane_tab,
                               pl.tabs, pl.table);
        else if (pl.L == 2 * TV)
            hipLaunchKernelGGL((fill_split_kernel<DT, 2 * TV, G>), dim3(pl.grid), dim3(64), 0, st,
                               planes, plane_stride, sidx, pl.nfull, pl.B, pl.rem, o, pl.lane_tab,
                               pl.tabs, pl.table);
        else
            return hipErrorInvalidValue;
    } else {
        hipLaunchKernelGGL((fill_leap_kernel<DT, G>), dim3(pl.grid), dim3(64), 0, st, planes,
                           plane_stride, sidx, pl.leap, o, pl.table);
    }
    return hipGetLastError();
}

template <class G>
static hipError_t launch_partition_d(const uint32_t *planes, uint64_t plane_stride, uint64_t sidx,
                                     int dtype, const PartitionLaunch &pl, void *out,
                                     hipStream_t st)
{
    switch (dtype) {
    case 0: return launch_partition_g<0, G>(planes, plane_stride, sidx, pl, out, st);
    case 1: return launch_partition_g<1, G>(planes, plane_stride, sidx, pl, out, st);
    default: return launch_partition_g<2, G>(planes, plane_stride, sidx, pl, out, st);
    }
}

hipError_t launch_partition(const uint32_t *planes, uint64_t plane_stride, uint64_t sidx,
                            int dtype, const PartitionLaunch &pl, void *out, int engine,
                            hipStream_t st)
{
    if (engine == 1) return launch_partition_d<GenF>(planes, plane_stride, sidx, dtype, pl, out, st);
    return launch_partition_d<GenI>(planes, plane_stride, sidx, dtype, pl, out, st);
}

}  // namespace mrg
