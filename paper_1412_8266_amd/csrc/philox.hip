// Philox4x32-10 stream sets (Salmon, Moraes, Dror & Shaw, SC 2011): the
// counter-based generator family the paper embeds beside MRG32k3a.  A stream's
// six state words are (position lo, hi, stream id lo, hi, key lo, hi); output
// number `position` is word position % 4 of the block whose 128-bit counter is
// (position / 4, stream id).  No jump tables: a jump adds to the position.
//
//   philox_init_kernel    stream g = g0 + s: position 0, id g, the set's key
//   philox_jump_kernel    position += e (per stream from device memory, or
//                         one e for the range)
//   philox_sm_kernel      stream-major fill: each thread about 16 4-value
//                         blocks of a row, consecutive threads on consecutive
//                         blocks, 16-byte stores when a block is aligned; row
//                         groups placed on the XCDs in the chunked order
//   philox_il_kernel      interleaved fill: one stream per lane, consecutive
//                         lanes write consecutive elements
// Fills do not move the positions; the host enqueues a uniform jump after them
// (a row's blocks are spread over several workgroups, which all read the
// position first).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gen_device.hpp"
#include "kernels.h"
#include "philox_device.h"  // philox10, philox_block, conversions

namespace mrg {
namespace {

// Conversions of a word: (2*(w>>9)+1)*2^-24 as binary32 (1 + k*2^-23 minus
// 1 - 2^-24, exact), (2w+1)*2^-33 as binary64 (one exact FMA).
template <int DT> struct PhiloxOut;
template <> struct PhiloxOut<0> {
    using T = uint32_t;
    __device__ static T conv(uint32_t w) { return w; }
};
template <> struct PhiloxOut<1> {
    using T = float;
    __device__ static T conv(uint32_t w) { return philox_to_f32(w); }
};
template <> struct PhiloxOut<2> {
    using T = double;
    __device__ static T conv(uint32_t w) { return philox_to_f64(w); }
};

__device__ __forceinline__ uint64_t position(const uint32_t *w)
{
    return (uint64_t)w[0] | (uint64_t)w[1] << 32;
}

__global__ void __launch_bounds__(256)
philox_init_kernel(uint32_t *__restrict__ planes, uint64_t plane_stride, uint64_t count,
                   uint64_t g0, uint64_t key)
{
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= count) return;
    const uint64_t g = g0 + s;
    const uint32_t w[6] = {0u, 0u, (uint32_t)g, (uint32_t)(g >> 32), (uint32_t)key,
                           (uint32_t)(key >> 32)};
    store_state(planes, plane_stride, s, w);
}

__global__ void __launch_bounds__(256)
philox_jump_kernel(uint32_t *__restrict__ planes, uint64_t plane_stride, uint64_t first,
                   uint64_t count, const uint64_t *__restrict__ exps, uint64_t e_uniform)
{
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= count) return;
    const uint64_t idx = first + s;
    const uint64_t e = exps ? exps[3 * s] : e_uniform;  // position wraps at 2^64
    const uint64_t pos = ((uint64_t)planes[idx] | (uint64_t)planes[plane_stride + idx] << 32) + e;
    planes[idx] = (uint32_t)pos;
    planes[plane_stride + idx] = (uint32_t)(pos >> 32);
}

// Stream-major: rows of n values, row s at out + s*n.  A workgroup of 256
// threads owns rpw rows, tpr = 256 / rpw threads each; thread j of a row
// writes blocks j, j + tpr, ... of the row (block b: the row's values
// [4b - off, 4b - off + 4) with off = position % 4).
template <int DT>
__global__ void __launch_bounds__(256)
philox_sm_kernel(const uint32_t *__restrict__ planes, uint64_t plane_stride, uint64_t first,
                 uint64_t count, uint64_t n, int rpw, unsigned char *__restrict__ out)
{
    using T = typename PhiloxOut<DT>::T;
    const int tpr = 256 / rpw;
    // several rows per workgroup: row groups in the chunked XCD order, so the
    // rows whose states share a state-plane line run on one XCD and each line
    // is fetched into one L2 (one row per workgroup keeps the dispatch order,
    // measured faster for such long rows)
    const uint64_t wg = rpw > 1 ? xcd_chunk(gridDim.x).first : blockIdx.x;
    const uint64_t s = wg * rpw + threadIdx.x / tpr;
    if (s >= count || (int)threadIdx.x >= rpw * tpr) return;
    uint32_t w[6];
    load_state(planes, plane_stride, first + s, w);
    const uint64_t pos = position(w);
    const uint64_t off = pos & 3, b0 = pos >> 2;
    const uint64_t nb = (off + n + 3) / 4;
    T *row = (T *)out + s * n;
    for (uint64_t b = threadIdx.x % tpr; b < nb; b += tpr) {
        uint32_t v[4];
        philox_block(w, b0 + b, v);
        const uint64_t k0 = 4 * b - off;  // row index of word 0 (wraps below 0 for b = 0)
        if (off == 0 && k0 + 4 <= n && ((uintptr_t)(row + k0) % (4 * sizeof(T))) == 0) {
            T *p = row + k0;
            if constexpr (DT == 2) {
                *(double2 *)p = make_double2(PhiloxOut<2>::conv(v[0]), PhiloxOut<2>::conv(v[1]));
                *(double2 *)(p + 2) = make_double2(PhiloxOut<2>::conv(v[2]), PhiloxOut<2>::conv(v[3]));
            } else {
                uint4 q;
                q.x = __builtin_bit_cast(uint32_t, PhiloxOut<DT>::conv(v[0]));
                q.y = __builtin_bit_cast(uint32_t, PhiloxOut<DT>::conv(v[1]));
                q.z = __builtin_bit_cast(uint32_t, PhiloxOut<DT>::conv(v[2]));
                q.w = __builtin_bit_cast(uint32_t, PhiloxOut<DT>::conv(v[3]));
                *(uint4 *)p = q;
            }
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint64_t k = k0 + j;  // below 0 wraps to a huge value: skipped
                if (k < n) row[k] = PhiloxOut<DT>::conv(v[j]);
            }
        }
    }
}

// Interleaved: out[k * count + s]; lane = stream, blocks in order.
template <int DT>
__global__ void __launch_bounds__(256)
philox_il_kernel(const uint32_t *__restrict__ planes, uint64_t plane_stride, uint64_t first,
                 uint64_t count, uint64_t n, unsigned char *__restrict__ out)
{
    using T = typename PhiloxOut<DT>::T;
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= count) return;
    uint32_t w[6];
    load_state(planes, plane_stride, first + s, w);
    const uint64_t pos = position(w);
    const uint64_t off = pos & 3, b0 = pos >> 2;
    const uint64_t nb = (off + n + 3) / 4;
    T *col = (T *)out + s;
    for (uint64_t b = 0; b < nb; ++b) {
        uint32_t v[4];
        philox_block(w, b0 + b, v);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint64_t k = 4 * b + j - off;
            if (k < n) col[k * count] = PhiloxOut<DT>::conv(v[j]);
        }
    }
}

unsigned grid256(uint64_t items) { return (unsigned)((items + 255) / 256); }

}  // namespace

hipError_t launch_philox_init(uint32_t *planes, uint64_t plane_stride, uint64_t count,
                              uint64_t g0, uint64_t key, hipStream_t st)
{
    hipLaunchKernelGGL(philox_init_kernel, dim3(grid256(count)), dim3(256), 0, st, planes,
                       plane_stride, count, g0, key);
    return hipGetLastError();
}

hipError_t launch_philox_jump(uint32_t *planes, uint64_t plane_stride, uint64_t first,
                              uint64_t count, const uint64_t *d_exp, uint64_t e, hipStream_t st)
{
    hipLaunchKernelGGL(philox_jump_kernel, dim3(grid256(count)), dim3(256), 0, st, planes,
                       plane_stride, first, count, d_exp, e);
    return hipGetLastError();
}

template <int DT>
static hipError_t launch_philox_fill_t(const uint32_t *planes, uint64_t plane_stride,
                                       uint64_t first, uint64_t count, uint64_t n, int layout,
                                       void *out, hipStream_t st)
{
    unsigned char *o = (unsigned char *)out;
    if (layout == 1) {
        hipLaunchKernelGGL((philox_il_kernel<DT>), dim3(grid256(count)), dim3(256), 0, st, planes,
                           plane_stride, first, count, n, o);
    } else {
        // threads per row: about 16 blocks each (a power of two, 1 .. 256), so
        // that each thread's state load and setup serve 64 values or more
        const uint64_t nb = (n + 6) / 4;
        int tpr = 1;
        while (tpr < 256 && (uint64_t)tpr * 16 < nb) tpr *= 2;
        const int rpw = 256 / tpr;
        const uint64_t wgs = (count + rpw - 1) / rpw;
        if (wgs > 0x7fffffffu) return hipErrorInvalidValue;
        hipLaunchKernelGGL((philox_sm_kernel<DT>), dim3((unsigned)wgs), dim3(256), 0, st, planes,
                           plane_stride, first, count, n, rpw, o);
    }
    return hipGetLastError();
}

hipError_t launch_philox_fill(const uint32_t *planes, uint64_t plane_stride, uint64_t first,
                              uint64_t count, uint64_t n, int dtype, int layout, void *out,
                              hipStream_t st)
{
    switch (dtype) {
    case 0: return launch_philox_fill_t<0>(planes, plane_stride, first, count, n, layout, out, st);
    case 1: return launch_philox_fill_t<1>(planes, plane_stride, first, count, n, layout, out, st);
    default: return launch_philox_fill_t<2>(planes, plane_stride, first, count, n, layout, out, st);
    }
}

}  // namespace mrg
