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
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mrg_arith.hpp"
#include "kernels.h"

namespace mrg {

// ---------------------------------------------------------------------------
// jump tables: T[c][w][d][9], c in {0,1}, w in [0,48), d in [0,16); d = 0 is
// the identity.  Exponent digit w of e (3 little-endian words) is
// (e >> 4w) & 15.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t exp_digit(uint64_t e0, uint64_t e1, uint64_t e2, int w)
{
    uint64_t word = w < 16 ? e0 : (w < 32 ? e1 : e2);
    return (uint32_t)(word >> (4 * (w & 15))) & 15u;
}

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

// ---------------------------------------------------------------------------
// generation
// ---------------------------------------------------------------------------
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
};

// Binary64 generator: centred integer-valued doubles, five FP64 operations
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
};

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

template <int DT, class G>
__device__ __forceinline__ void put1(unsigned char *p, G &g)
{
    if constexpr (DT == 0) *(uint32_t *)p = g.next_u32();
    else if constexpr (DT == 1) *(float *)p = g.next_f32();
    else *(double *)p = g.next_f64();
}

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

// One wave (64 lanes) per workgroup; lane = stream.  Each full tile of TV
// values per stream is generated into the lane's LDS row and written back
// as 16-byte chunks, LPR lanes per row, so every store instruction covers
// RPI rows x TB contiguous bytes.  The LDS row pitch TB+16 keeps both the
// b128 writes (lanes on different rows) and the reads (lanes along a row)
// free of bank conflicts.
template <int DT, int TB, class G>
__global__ void __launch_bounds__(64)
fill_sm_kernel(uint32_t *__restrict__ planes, uint64_t plane_stride, uint64_t first,
               uint64_t count, uint64_t n, unsigned char *__restrict__ out, int vec_ok)
{
    constexpr int ES = Elem<DT>::size;
    constexpr int TV = TB / ES;      // values per row per tile
    constexpr int RS = TB + 16;      // LDS row pitch (bytes)
    constexpr int LPR = TB / 16;     // lanes per row when flushing
    constexpr int RPI = 64 / LPR;    // rows per flush instruction
    constexpr int NJ = 64 / RPI;     // flush instructions per tile
    __shared__ __attribute__((aligned(16))) unsigned char lds[64 * RS];

    const int lane = threadIdx.x;
    const uint64_t s0 = (uint64_t)blockIdx.x * 64;
    const uint64_t nrows = count - s0 < 64 ? count - s0 : 64;
    const bool active = (uint64_t)lane < nrows;
    const uint64_t idx = first + s0 + lane;

    uint32_t w[6] = {1u, 1u, 1u, 1u, 1u, 1u};
    if (active) load_state(planes, plane_stride, idx, w);
    G g;
    g.load(w);

    const uint64_t row_bytes = n * ES;
    unsigned char *my_lds = lds + lane * RS;
    // rows this lane flushes: r_j = lane / LPR + RPI * j, chunk lane % LPR
    const int chunk = lane % LPR;
    unsigned char *rowp[NJ];
    bool rowa[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int r = lane / LPR + RPI * j;
        rowa[j] = (uint64_t)r < nrows;
        rowp[j] = out + (s0 + r) * row_bytes + chunk * 16;
    }

    const uint64_t nfull = n / TV;
    for (uint64_t t = 0; t < nfull; ++t) {
#pragma unroll
        for (int c = 0; c < TB / 16; ++c)
            *(uint4 *)(my_lds + c * 16) = gen16<DT>(g);
        __syncthreads();
        const uint64_t off = t * TB;
        if (vec_ok) {
            // all LDS reads first, one wait, then the stores
            uint4 v[NJ];
#pragma unroll
            for (int j = 0; j < NJ; ++j)
                v[j] = *(const uint4 *)(lds + (lane / LPR + RPI * j) * RS + chunk * 16);
            if (nrows == 64) {
#pragma unroll
                for (int j = 0; j < NJ; ++j) *(uint4 *)(rowp[j] + off) = v[j];
            } else {
#pragma unroll
                for (int j = 0; j < NJ; ++j)
                    if (rowa[j]) *(uint4 *)(rowp[j] + off) = v[j];
            }
        } else {
            // element stores: lane e covers (row e / TV, col e % TV)
            for (int e = lane; e < 64 * TV; e += 64) {
                const int r = e / TV, col = e % TV;
                if ((uint64_t)r < nrows) {
                    unsigned char *dst = out + (s0 + r) * row_bytes + off + (uint64_t)col * ES;
                    const unsigned char *src = lds + r * RS + col * ES;
                    if constexpr (ES == 4) *(uint32_t *)dst = *(const uint32_t *)src;
                    else *(uint64_t *)dst = *(const uint64_t *)src;
                }
            }
        }
        __syncthreads();
    }
    // tail: fewer than TV values per row
    const int tail = (int)(n - nfull * TV);
    if (tail) {
        for (int c = 0; c < tail; ++c) put1<DT>(my_lds + c * ES, g);
        __syncthreads();
        const uint64_t off = nfull * TB;
        for (int e = lane; e < 64 * tail; e += 64) {
            const int r = e / tail, col = e % tail;
            if ((uint64_t)r < nrows) {
                unsigned char *dst = out + (s0 + r) * row_bytes + off + (uint64_t)col * ES;
                const unsigned char *src = lds + r * RS + col * ES;
                if constexpr (ES == 4) *(uint32_t *)dst = *(const uint32_t *)src;
                else *(uint64_t *)dst = *(const uint64_t *)src;
            }
        }
    }
    if (active) {
        g.store(w);
        store_state(planes, plane_stride, idx, w);
    }
}

// Interleaved output out[k * count + s]: consecutive lanes are consecutive
// streams, so each step is one coalesced store per wave.
template <int DT, class G>
__global__ void __launch_bounds__(256)
fill_il_kernel(uint32_t *__restrict__ planes, uint64_t plane_stride, uint64_t first,
               uint64_t count, uint64_t n, unsigned char *__restrict__ out)
{
    constexpr int ES = Elem<DT>::size;
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= count) return;
    const uint64_t idx = first + s;
    uint32_t w[6];
    load_state(planes, plane_stride, idx, w);
    G g;
    g.load(w);
    unsigned char *p = out + s * ES;
    const uint64_t step = count * ES;
    uint64_t k = 0;
    for (; k + 4 <= n; k += 4) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            put1<DT>(p, g);
            p += step;
        }
    }
    for (; k < n; ++k) {
        put1<DT>(p, g);
        p += step;
    }
    g.store(w);
    store_state(planes, plane_stride, idx, w);
}

// Stream-major output with one wave per stream (sequence splitting inside the
// stream, sec. 2.3): the stream's n outputs are cut into chunks of 64*L
// values and lane l generates the L consecutive values [l*L, l*L + L) of each
// chunk, starting from A^(l*L) applied to the chunk's first state
// (lane_tab[l], formed on the host).  The next chunk starts where lane 63
// ended.  Every LDS flush then writes 64 pieces of 128 bytes that tile the
// chunk's 64*L*ES contiguous bytes, so the HBM write stream is nearly
// sequential.  The end state A^n * state (Mn) is written back by lane 0.
// Workgroups stride over the streams so that the streams in flight stay
// adjacent in memory.
template <int DT, int L, class G>
__global__ void __launch_bounds__(64)
fill_coop_kernel(uint32_t *__restrict__ planes, uint64_t plane_stride, uint64_t first,
                 uint64_t count, uint64_t n, unsigned char *__restrict__ out, int vec_ok,
                 const uint32_t *__restrict__ lane_tab, JumpMatrices Mn)
{
    constexpr int ES = Elem<DT>::size;
    constexpr int TV = 128 / ES;   // values per 128-byte piece
    constexpr int NH = L / TV;     // pieces per lane per chunk
    constexpr int RS = 128 + 16;   // LDS row pitch (bytes)
    static_assert(NH >= 1 && L % TV == 0, "chunk must be whole pieces");
    __shared__ __attribute__((aligned(16))) unsigned char lds[64 * RS];

    const int lane = threadIdx.x;
    uint32_t m[18];
#pragma unroll
    for (int i = 0; i < 18; ++i) m[i] = lane_tab[lane * 18 + i];
    unsigned char *my_lds = lds + lane * RS;
    const uint64_t chunk_vals = (uint64_t)64 * L;
    const uint64_t nchunks = (n + chunk_vals - 1) / chunk_vals;
    const int prow = lane >> 3;        // flush: 8 lanes per 128-byte piece
    const int pcol = (lane & 7) * 16;  //        8 pieces per instruction

    // whole chunks only: the end state is lane 63's after the last chunk;
    // otherwise it is A^n * state, computed up front
    const bool whole = n % chunk_vals == 0;

    for (uint64_t s = blockIdx.x; s < count; s += gridDim.x) {
        const uint64_t idx = first + s;
        uint32_t w[6];
        load_state(planes, plane_stride, idx, w);
        uint32_t fin[6] = {w[0], w[1], w[2], w[3], w[4], w[5]};
        if (!whole) {
            matvec3<C1>(Mn.m, fin[0], fin[1], fin[2]);
            matvec3<C2>(Mn.m + 9, fin[3], fin[4], fin[5]);
        }
        unsigned char *srow = out + s * n * ES;

        for (uint64_t c = 0; c < nchunks; ++c) {
            uint32_t st[6] = {w[0], w[1], w[2], w[3], w[4], w[5]};
            matvec3<C1>(m, st[0], st[1], st[2]);
            matvec3<C2>(m + 9, st[3], st[4], st[5]);
            G g;
            g.load(st);
            const uint64_t v0 = c * chunk_vals;
            const bool full = v0 + chunk_vals <= n;
            for (int h = 0; h < NH; ++h) {
#pragma unroll
                for (int q = 0; q < 8; ++q) *(uint4 *)(my_lds + q * 16) = gen16<DT>(g);
                __syncthreads();
                if (full && vec_ok) {
                    uint4 v[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j)
                        v[j] = *(const uint4 *)(lds + (prow + 8 * j) * RS + pcol);
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const uint64_t pos = v0 + (uint64_t)(prow + 8 * j) * L + h * TV;
                        *(uint4 *)(srow + pos * ES + pcol) = v[j];
                    }
                } else {
                    for (int e = lane; e < 64 * TV; e += 64) {
                        const int r = e / TV, i = e % TV;
                        const uint64_t pos = v0 + (uint64_t)r * L + h * TV + i;
                        if (pos < n) {
                            const unsigned char *src = lds + r * RS + i * ES;
                            if constexpr (ES == 4) *(uint32_t *)(srow + pos * ES) = *(const uint32_t *)src;
                            else *(uint64_t *)(srow + pos * ES) = *(const uint64_t *)src;
                        }
                    }
                }
                __syncthreads();
            }
            if (c + 1 < nchunks) {  // chunk c was full: lane 63 ends at the next chunk's start
                uint32_t e[6];
                g.store(e);
#pragma unroll
                for (int k = 0; k < 6; ++k) w[k] = __shfl(e[k], 63);
            } else if (whole) {
                g.store(fin);
            }
        }
        if (lane == (whole ? 63 : 0)) store_state(planes, plane_stride, idx, fin);
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
                                uint64_t count, uint64_t n, int layout, void *out, int vec_ok,
                                const FillLaunch &fl, int tile_bytes, hipStream_t st)
{
    unsigned char *o = (unsigned char *)out;
    if (layout == 1) {
        hipLaunchKernelGGL((fill_il_kernel<DT, G>), dim3(grid_of(count, 256)), dim3(256), 0, st,
                           planes, plane_stride, first, count, n, o);
    } else if (fl.kernel == 1) {
        const dim3 grid(fl.grid), block(64);
        if (fl.L == 64 && DT != 2)
            hipLaunchKernelGGL((fill_coop_kernel<DT, 64, G>), grid, block, 0, st, planes,
                               plane_stride, first, count, n, o, vec_ok, fl.lane_tab, fl.Mn);
        else if (fl.L == 32)
            hipLaunchKernelGGL((fill_coop_kernel<DT, 32, G>), grid, block, 0, st, planes,
                               plane_stride, first, count, n, o, vec_ok, fl.lane_tab, fl.Mn);
        else if (fl.L == 16 && DT == 2)
            hipLaunchKernelGGL((fill_coop_kernel<2, 16, G>), grid, block, 0, st, planes,
                               plane_stride, first, count, n, o, vec_ok, fl.lane_tab, fl.Mn);
        else
            return hipErrorInvalidValue;
    } else if (tile_bytes >= 256) {
        hipLaunchKernelGGL((fill_sm_kernel<DT, 256, G>), dim3(grid_of(count, 64)), dim3(64), 0, st,
                           planes, plane_stride, first, count, n, o, vec_ok);
    } else {
        hipLaunchKernelGGL((fill_sm_kernel<DT, 128, G>), dim3(grid_of(count, 64)), dim3(64), 0, st,
                           planes, plane_stride, first, count, n, o, vec_ok);
    }
    return hipGetLastError();
}

template <class G>
static hipError_t launch_fill_d(uint32_t *planes, uint64_t plane_stride, uint64_t first,
                                uint64_t count, uint64_t n, int dtype, int layout, void *out,
                                int vec_ok, const FillLaunch &fl, int tile_bytes, hipStream_t st)
{
    switch (dtype) {
    case 0: return launch_fill_g<0, G>(planes, plane_stride, first, count, n, layout, out, vec_ok, fl, tile_bytes, st);
    case 1: return launch_fill_g<1, G>(planes, plane_stride, first, count, n, layout, out, vec_ok, fl, tile_bytes, st);
    default: return launch_fill_g<2, G>(planes, plane_stride, first, count, n, layout, out, vec_ok, fl, tile_bytes, st);
    }
}

hipError_t launch_fill(uint32_t *planes, uint64_t plane_stride, uint64_t first, uint64_t count,
                       uint64_t n, int dtype, int layout, void *out, int vec_ok,
                       const FillLaunch &fl, const FillTuning &tune, hipStream_t st)
{
    if (tune.engine == 1)
        return launch_fill_d<GenF>(planes, plane_stride, first, count, n, dtype, layout, out,
                                   vec_ok, fl, tune.tile_bytes, st);
    return launch_fill_d<GenI>(planes, plane_stride, first, count, n, dtype, layout, out, vec_ok,
                               fl, tune.tile_bytes, st);
}

}  // namespace mrg
