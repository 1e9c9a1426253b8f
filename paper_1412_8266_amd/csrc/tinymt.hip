// TinyMT32 stream sets: the paper's hybrid for the Mersenne-Twister family
// (sec. 4.2).  Threads of a group share one parameter set; each thread draws
// from its own sub-stream of that generator, the sequence being cut into
// chunks of 2^64 outputs (sequence splitting, sec. 2.3).  A stream's six
// state words are (s0, s1, s2, s3, q, 0), q the global index of its
// parameter set; each set has a device record (parameters, characteristic
// polynomial, table of x^(2^i) mod phi), tinymt_arith.hpp.
//
//   tmt_candidates_kernel  parameter search: one candidate per thread,
//                          Berlekamp-Massey then Rabin's test
//   tmt_records_kernel     one parameter set per thread: check it, build
//                          its record
//   tmt_init_kernel        stream g: set g / per_param seeded, jumped
//                          (g % per_param) * 2^64
//   tmt_jump_kernel        per-stream or uniform polynomial jumps
//   tmt_sm_kernel          stream-major fill: one stream per lane, rows
//                          staged in LDS and written as 16-byte line pieces
//   tmt_il_kernel          interleaved fill: one stream per lane,
//                          consecutive lanes write consecutive elements
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gen_device.hpp"   // rows_fill, rows_fill_carry, rows_fill_short, put1
#include "kernels.h"
#include "tinymt_device.h"

namespace mrg {
namespace {

__global__ void __launch_bounds__(64)
tmt_candidates_kernel(uint64_t master, uint64_t c0, uint64_t n, uint32_t *__restrict__ flags,
                      uint32_t *__restrict__ phis)
{
    const uint64_t i = (uint64_t)blockIdx.x * 64 + threadIdx.x;
    if (i >= n) return;
    uint32_t p[3], phi[4];
    tmt::candidate(master, c0 + i, p);
    const int L = tmt::charpoly(p, phi);
    const bool ok = L == 127 && tmt::irreducible127(phi);
    flags[i] = (uint32_t)L | (ok ? 1u << 16 : 0u);
    if (phis) {
#pragma unroll
        for (int k = 0; k < 4; ++k) phis[4 * i + k] = phi[k];
    }
}

// params [n][3] -> records [n][kRecordWords]; ok[i] = 1 when set i has a
// degree-127 irreducible characteristic polynomial.
__global__ void __launch_bounds__(64)
tmt_records_kernel(const uint32_t *__restrict__ params, uint64_t n, uint32_t *__restrict__ records,
                   uint32_t *__restrict__ ok)
{
    const uint64_t i = (uint64_t)blockIdx.x * 64 + threadIdx.x;
    if (i >= n) return;
    const uint32_t p[3] = {params[3 * i], params[3 * i + 1], params[3 * i + 2]};
    uint32_t phi[4];
    const bool good = tmt::params_ok(p, phi);
    uint32_t *rec = records + i * tmt::kRecordWords;
    rec[0] = p[0];
    rec[1] = p[1];
    rec[2] = p[2];
    rec[3] = 0u;
#pragma unroll
    for (int k = 0; k < 4; ++k) rec[tmt::kRecPhi + k] = phi[k];
    if (good) tmt::pow_table(phi, rec + tmt::kRecPow);
    ok[i] = good ? 1u : 0u;
}

__global__ void __launch_bounds__(256)
tmt_init_kernel(uint32_t *__restrict__ planes, uint64_t plane_stride, uint64_t count, uint64_t g0,
                uint64_t per_param, uint64_t q0, uint64_t master,
                const uint32_t *__restrict__ records)
{
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= count) return;
    const uint64_t g = g0 + s, q = g / per_param, j = g % per_param;
    const uint32_t *rec = records + (q - q0) * tmt::kRecordWords;
    const uint32_t mat1 = rec[0], mat2 = rec[1], tmat = rec[2];
    uint32_t st[4];
    tmt::seed_status(tmt::set_seed(master, q), mat1, mat2, tmat, st);
    tmt::jump(st, mat1, mat2, rec + tmt::kRecPhi, rec + tmt::kRecPow, 0, j, 0);
    const uint32_t w[6] = {st[0], st[1], st[2], st[3], (uint32_t)q, 0u};
    store_state(planes, plane_stride, s, w);
}

__global__ void __launch_bounds__(256)
tmt_jump_kernel(uint32_t *__restrict__ planes, uint64_t plane_stride, uint64_t first,
                uint64_t count, const uint64_t *__restrict__ exps, uint64_t e0, uint64_t e1,
                uint64_t e2, const uint32_t *__restrict__ records, uint64_t q0)
{
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= count) return;
    if (exps) {
        e0 = exps[3 * s];
        e1 = exps[3 * s + 1];
        e2 = exps[3 * s + 2];
    }
    TinyMTStream r;
    r.load(planes, plane_stride, first + s, records, q0);
    r.jump(e0, e1, e2);
    r.store(planes, plane_stride, first + s);
}

// Stream-major: rows of n values, row s at out + s*n; one wave of 64 lanes
// per 64 rows (lanes past the last row draw from a dummy state and write
// nothing).
template <int DT, int TB>
__global__ void __launch_bounds__(64)
tmt_sm_kernel(uint32_t *__restrict__ planes, uint64_t plane_stride, uint64_t first,
              uint64_t count, uint64_t n, unsigned char *__restrict__ out,
              const uint32_t *__restrict__ records, uint64_t q0)
{
    constexpr int ES = Elem<DT>::size;
    // TB = 0: rows off their lines, written by rows_fill_carry in 128-byte windows
    __shared__ __attribute__((aligned(16))) unsigned char lds[64 * (TB ? TB + 16 : 128 + 160)];
    const int lane = threadIdx.x;
    const uint64_t s0 = (uint64_t)blockIdx.x * 64;
    const uint64_t nrows = count - s0 < 64 ? count - s0 : 64;
    const bool active = (uint64_t)lane < nrows;
    TinyMTStream g;
    if (active) {
        g.load(planes, plane_stride, first + s0 + lane, records, q0);
    } else {
        g.s0 = g.s1 = g.s2 = g.s3 = 1u;
        g.q = 0u;
        g.mat1 = g.mat2 = g.tmat = 0u;
        g.rec = records;
    }
    if (n * ES < 128) {  // the wave's rows are one block shorter than 64 lines
        rows_fill_short<DT, TinyMTStream>(g, lds, lane, nrows, out + s0 * n * ES, n);
    } else {
        if constexpr (TB == 0)
            rows_fill_carry<DT, 128, TinyMTStream>(g, lds, lane, nrows, out + s0 * n * ES, n);
        else
            rows_fill<DT, TB, TinyMTStream>(g, lds, lane, nrows, out + s0 * n * ES, n * ES, n);
    }
    if (active) g.store(planes, plane_stride, first + s0 + lane);
}

// Interleaved output out[k * count + s].
template <int DT>
__global__ void __launch_bounds__(256)
tmt_il_kernel(uint32_t *__restrict__ planes, uint64_t plane_stride, uint64_t first,
              uint64_t count, uint64_t n, unsigned char *__restrict__ out,
              const uint32_t *__restrict__ records, uint64_t q0)
{
    constexpr int ES = Elem<DT>::size;
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= count) return;
    TinyMTStream g;
    g.load(planes, plane_stride, first + s, records, q0);
    unsigned char *p = out + s * ES;
    const uint64_t step = count * ES;
    uint64_t k = 0;
    for (; k + 4 <= n; k += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            put1<DT>(p, g);
            p += step;
        }
    }
    for (; k < n; ++k) {
        put1<DT>(p, g);
        p += step;
    }
    g.store(planes, plane_stride, first + s);
}

unsigned blocks_of(uint64_t items, unsigned per) { return (unsigned)((items + per - 1) / per); }

template <int DT>
hipError_t launch_tmt_fill_t(uint32_t *planes, uint64_t plane_stride, uint64_t first,
                             uint64_t count, uint64_t n, int layout, void *out,
                             const uint32_t *records, uint64_t q0, int tile_bytes, hipStream_t st)
{
    unsigned char *o = (unsigned char *)out;
    if (layout == 1) {
        hipLaunchKernelGGL((tmt_il_kernel<DT>), dim3(blocks_of(count, 256)), dim3(256), 0, st,
                           planes, plane_stride, first, count, n, o, records, q0);
    } else {
        constexpr int ES = Elem<DT>::size;
        const int tb = tile_bytes ? tile_bytes : (n * ES < 1024 ? 128 : 256);
        if (!tile_bytes && ((uintptr_t)out % 128 || (n * ES) % 128))
            // rows off their lines: one write per shared line (rows_fill_carry)
            hipLaunchKernelGGL((tmt_sm_kernel<DT, 0>), dim3(blocks_of(count, 64)), dim3(64), 0,
                               st, planes, plane_stride, first, count, n, o, records, q0);
        else if (tb == 128)
            hipLaunchKernelGGL((tmt_sm_kernel<DT, 128>), dim3(blocks_of(count, 64)), dim3(64), 0,
                               st, planes, plane_stride, first, count, n, o, records, q0);
        else
            hipLaunchKernelGGL((tmt_sm_kernel<DT, 256>), dim3(blocks_of(count, 64)), dim3(64), 0,
                               st, planes, plane_stride, first, count, n, o, records, q0);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_tmt_candidates(uint64_t master, uint64_t c0, uint64_t n, uint32_t *flags,
                                 uint32_t *phis, hipStream_t st)
{
    hipLaunchKernelGGL(tmt_candidates_kernel, dim3(blocks_of(n, 64)), dim3(64), 0, st, master, c0,
                       n, flags, phis);
    return hipGetLastError();
}

hipError_t launch_tmt_records(const uint32_t *params, uint64_t n, uint32_t *records, uint32_t *ok,
                              hipStream_t st)
{
    hipLaunchKernelGGL(tmt_records_kernel, dim3(blocks_of(n, 64)), dim3(64), 0, st, params, n,
                       records, ok);
    return hipGetLastError();
}

hipError_t launch_tmt_init(uint32_t *planes, uint64_t plane_stride, uint64_t count, uint64_t g0,
                           uint64_t per_param, uint64_t q0, uint64_t master,
                           const uint32_t *records, hipStream_t st)
{
    hipLaunchKernelGGL(tmt_init_kernel, dim3(blocks_of(count, 256)), dim3(256), 0, st, planes,
                       plane_stride, count, g0, per_param, q0, master, records);
    return hipGetLastError();
}

hipError_t launch_tmt_jump(uint32_t *planes, uint64_t plane_stride, uint64_t first, uint64_t count,
                           const uint64_t *d_exp, const uint64_t e[3], const uint32_t *records,
                           uint64_t q0, hipStream_t st)
{
    hipLaunchKernelGGL(tmt_jump_kernel, dim3(blocks_of(count, 256)), dim3(256), 0, st, planes,
                       plane_stride, first, count, d_exp, e[0], e[1], e[2], records, q0);
    return hipGetLastError();
}

hipError_t launch_tmt_fill(uint32_t *planes, uint64_t plane_stride, uint64_t first, uint64_t count,
                           uint64_t n, int dtype, int layout, void *out, const uint32_t *records,
                           uint64_t q0, int tile_bytes, hipStream_t st)
{
    switch (dtype) {
    case 0: return launch_tmt_fill_t<0>(planes, plane_stride, first, count, n, layout, out,
                                        records, q0, tile_bytes, st);
    case 1: return launch_tmt_fill_t<1>(planes, plane_stride, first, count, n, layout, out,
                                        records, q0, tile_bytes, st);
    default: return launch_tmt_fill_t<2>(planes, plane_stride, first, count, n, layout, out,
                                         records, q0, tile_bytes, st);
    }
}

}  // namespace mrg
