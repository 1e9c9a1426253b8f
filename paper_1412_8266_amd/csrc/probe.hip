// Store-only probes: the write bandwidth HBM grants to a store pattern, with
// no generation work, so that the fill kernels can be compared with what the
// same stores alone attain.
//   pattern 0: streaming 16-byte stores, one per thread, consecutive lanes
//              and workgroups on consecutive addresses, so the front of
//              writes moves through memory in one pass (each wave
//              instruction covers 1 KiB);
//   pattern 1: the wave-per-stream fill's geometry at 16 lanes per stream and
//              256 uint32 per lane (4 rows of 16 KiB per wave): each flush
//              stages two 128-byte pieces per lane (adjacent lines of its
//              1 KiB member segment) in LDS and writes them as 16-byte stores,
//              each instruction four runs of two lines 1 KiB apart in a row;
//   pattern 2: the same 64 KiB per wave written as runs of 8 consecutive
//              lines (1 KiB) per instruction, one run per 1 KiB member
//              segment: what eight pieces per lane per flush would attain;
//   pattern 3: as pattern 1 with one piece per lane per flush (8 single
//              lines 1 KiB apart per instruction).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace mrg {

__global__ void __launch_bounds__(256) probe_stream_kernel(uint4 *__restrict__ out, uint64_t n16)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint32_t tag = threadIdx.x * 0x9E3779B9u;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        out[i] = make_uint4(tag, (uint32_t)i, tag ^ 1u, (uint32_t)(i >> 32));
}

// NP pieces per lane per flush: store j takes piece P = 8j + prow, piece
// P % NP of lane P / NP (stream (P / NP) / 16, member (P / NP) % 16).
template <int NP>
__global__ void __launch_bounds__(64) probe_pieces_kernel(unsigned char *__restrict__ out,
                                                          uint64_t groups)
{
    constexpr int RS = NP * 128 + 16, L_BYTES = 1024, ROW = 16384;
    __shared__ __attribute__((aligned(16))) unsigned char lds[64 * RS];
    const int lane = threadIdx.x;
    const int prow = lane >> 3, pcol = (lane & 7) * 16;
    for (uint64_t grp = blockIdx.x; grp < groups; grp += gridDim.x) {
        unsigned char *base = out + grp * 4 * ROW;
        for (int h = 0; h < 8; h += NP) {
#pragma unroll
            for (int p = 0; p < NP; ++p)
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    *(uint4 *)(lds + lane * RS + p * 128 + q * 16) =
                        make_uint4((uint32_t)grp, (uint32_t)(h + p), (uint32_t)lane, (uint32_t)q);
            __syncthreads();
            uint4 v[8 * NP];
#pragma unroll
            for (int j = 0; j < 8 * NP; ++j) {
                const int P = 8 * j + prow;
                v[j] = *(const uint4 *)(lds + (P / NP) * RS + (P % NP) * 128 + pcol);
            }
#pragma unroll
            for (int j = 0; j < 8 * NP; ++j) {
                const int P = 8 * j + prow, owner = P / NP;
                const int t = owner / 16, g = owner % 16;
                *(uint4 *)(base + t * ROW + g * L_BYTES + (h + P % NP) * 128 + pcol) = v[j];
            }
            __syncthreads();
        }
    }
}

__global__ void __launch_bounds__(64) probe_runs_kernel(unsigned char *__restrict__ out,
                                                        uint64_t groups)
{
    const int lane = threadIdx.x, p = lane >> 3, col = (lane & 7) * 16;
    for (uint64_t grp = blockIdx.x; grp < groups; grp += gridDim.x) {
        unsigned char *base = out + grp * 65536;
        const uint4 v = make_uint4((uint32_t)grp, (uint32_t)lane, 0x5A5Au, 0xA5A5u);
#pragma unroll
        for (int q = 0; q < 64; ++q)  // member segment q, its 8 lines
            *(uint4 *)(base + q * 1024 + p * 128 + col) = v;
    }
}

hipError_t launch_write_probe(void *out, uint64_t bytes, int pattern, hipStream_t st)
{
    if (pattern == 0) {
        const uint64_t n16 = bytes / 16;
        const uint64_t blocks = (n16 + 255) / 256;
        const unsigned grid = (unsigned)(blocks < 0x7fffffffu ? blocks : 0x7fffffffu);
        hipLaunchKernelGGL(probe_stream_kernel, dim3(grid), dim3(256), 0, st, (uint4 *)out, n16);
    } else if (pattern == 2) {
        const uint64_t groups = bytes / 65536;
        const unsigned grid = (unsigned)(groups < (1u << 30) ? groups : (1u << 30));
        hipLaunchKernelGGL(probe_runs_kernel, dim3(grid), dim3(64), 0, st, (unsigned char *)out,
                           groups);
    } else {
        const uint64_t groups = bytes / (4 * 16384);
        const unsigned grid = (unsigned)(groups < (1u << 30) ? groups : (1u << 30));
        if (pattern == 3)
            hipLaunchKernelGGL(probe_pieces_kernel<1>, dim3(grid), dim3(64), 0, st,
                               (unsigned char *)out, groups);
        else
            hipLaunchKernelGGL(probe_pieces_kernel<2>, dim3(grid), dim3(64), 0, st,
                               (unsigned char *)out, groups);
    }
    return hipGetLastError();
}

}  // namespace mrg
