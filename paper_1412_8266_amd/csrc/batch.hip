// Persistent batched generation: many fill requests of uneven stream counts
// and lengths in a few persistent launches.
//
// Each request is cut into work items of one wave:
//   - a wave item is one segment [v0, v1) of one stream, written with
//     wave_fill (lane l owns consecutive L-value pieces); the segment's first
//     state is the stream's state jumped by v0 with the windowed tables
//     (sequence splitting inside a stream, sec. 2.3);
//   - a row item is up to 16 blocks of up to 64 streams of a short-stream
//     request, one stream per lane, each block written with rows_fill_short,
//     rows_fill_carry_w or rows_fill.
// One launch per group (batch.h): wave items of one dtype, or the row items
// of every dtype, largest first, followed by the wave items of one dtype.
// Persistent workgroups (one wave each) claim items from a global counter or
// take them round robin; item i belongs to the request r with
// prefix[r] <= i < prefix[r+1].  A request in substream mode draws its streams
// from one stream: stream j is substream sub0 + j, i.e. that stream's state
// jumped by (sub0 + j) * 2^76 (sec. 4.1), and leaves the state unchanged.
// Otherwise each stream's end state is written back: in place when one item
// covers the stream, else to a scratch slot that batch_copyback_kernel moves
// to the state planes after the persistent kernel (a later segment of the
// same stream may still be reading the old state).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "batch.h"
#include "gen_device.hpp"

namespace mrg {

__global__ void batch_reset_kernel(unsigned long long *counter) { *counter = 0ull; }

// r with prefix[r] <= item < prefix[r+1] (prefix strictly increasing over
// [0, nreq], item wave-uniform): a 64-way search, one probe per lane, so a
// group of up to 4096 requests takes two dependent loads.
__device__ __forceinline__ uint32_t find_req(const uint64_t *__restrict__ prefix, uint32_t nreq,
                                             uint64_t item, int lane)
{
    uint32_t lo = 0, hi = nreq;  // prefix[lo] <= item < prefix[hi]
    for (;;) {
        const uint32_t step = hi - lo > 64 ? (hi - lo + 63) / 64 : 1;
        const uint32_t idx = lo + (uint32_t)lane * step;
        const bool le = idx < hi && prefix[idx] <= item;
        const uint32_t cnt = (uint32_t)__popcll(__ballot(le));  // le holds on a prefix of lanes
        lo += (cnt - 1) * step;
        if (step == 1) return lo;
        hi = lo + step < hi ? lo + step : hi;
    }
}

// Lane 0's value in a scalar register, so that everything derived from it
// (request index, descriptor fields, addresses) stays wave-uniform: scalar
// loads, and no vector registers spent on it.
__device__ __forceinline__ uint64_t lane0_uniform(uint64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

template <int DT, class G>
__device__ __forceinline__ void wave_item(const BatchReq &R, uint64_t local, unsigned char *lds,
                                          int lane, const uint32_t *m, const BatchArgs &A)
{
    constexpr int ES = Elem<DT>::size;
    constexpr int L = kBatchLaneBytes / ES;  // values per lane per chunk
    const bool subs = R.flags & kReqSubstreams;
    uint64_t j0, j1, q;  // streams [j0, j1), segment q of each
    if (R.spi > 1) {
        j0 = local * R.spi;
        j1 = j0 + R.spi < R.k ? j0 + R.spi : R.k;
        q = 0;
    } else {
        j0 = local / R.segs;
        j1 = j0 + 1;
        q = local % R.segs;
    }
    const uint64_t v0 = q * R.seg;
    const uint64_t v1 = v0 + R.seg < R.n ? v0 + R.seg : R.n;
    for (uint64_t j = j0; j < j1; ++j) {
        uint32_t w[6];
        load_state(A.planes, A.plane_stride, subs ? R.stream0 : R.stream0 + j, w);
        const uint64_t sub = subs ? R.sub0 + j : 0;
        // exponent v0 + sub * 2^76 (v0 < 2^64: no carry between the words)
        jump_global(A.table, v0, sub << 12, sub >> 52, 0, kTableWindows, w);
        const bool end = (R.flags & kReqWriteBack) && v1 == R.n;
        wave_fill<DT, L, G, false, 64, 0, 2>(w, m, lds, lane, R.out + j * R.n * ES, 0, 1, v0, v1,
                                             A.table, A.lane_tab, end);
        if (end) {
            if (lane == 0) {
                if (R.segs == 1) store_state(A.planes, A.plane_stride, R.stream0 + j, w);
                else store_state(A.scratch, A.scratch_stride, R.scratch0 + j, w);
            }
        }
    }
}

template <int DT, class G>
__device__ __forceinline__ void row_block(const BatchReq &R, uint64_t r0, unsigned char *lds, int lane,
                                          const BatchArgs &A)
{
    constexpr int ES = Elem<DT>::size;
    const uint64_t nrows = R.k - r0 < 64 ? R.k - r0 : 64;
    const bool active = (uint64_t)lane < nrows;
    const uint64_t j = r0 + lane;
    const bool subs = R.flags & kReqSubstreams;
    // one stream per lane, as a user kernel draws (public Stream object)
    Stream<G> s;
    if (active) {
        s.load(A.planes, A.plane_stride, subs ? R.stream0 : R.stream0 + j);
    } else {
        const uint32_t dummy[6] = {1u, 1u, 1u, 1u, 1u, 1u};
        s.g.load(dummy);
    }
    if (subs) s.substream(A.table, active ? R.sub0 + j : 0);
    unsigned char *out0 = R.out + r0 * R.n * ES;
    if (R.n * ES < 128)
        // the item's rows are one block shorter than 64 lines
        rows_fill_short<DT, G>(s.g, lds, lane, nrows, out0, R.n);
    else if ((uintptr_t)out0 % 128 || (R.n * ES) % 128)
        // rows off their lines: one write per line shared by two rows
        // (dword staging only: the 16-byte variant's registers on top of the
        // other paths of this kernel would spill)
        rows_fill_carry_w<DT, 128, G, false>(s.g, lds, lane, nrows, out0, R.n);
    else
        rows_fill<DT, 128, G, false>(s.g, lds, lane, nrows, out0, R.n * ES, R.n);
    if ((R.flags & kReqWriteBack) && active) s.store(A.planes, A.plane_stride, R.stream0 + j);
}

// One persistent kernel per group: wave items of dtype DT, led in the first
// group (KIND = kKindRows) by the row items of every dtype.  The writers move each LDS
// piece straight to memory (READ_ALL = false): staging all eight pieces in an
// array first, as the plain fill kernels do, sends that array to scratch
// memory inside this loop.  Wave items stage two pieces per member per flush
// (runs of two lines per store instruction), row items one 128-byte window
// per row and its spill (rows_fill_carry): 17-18 KiB of LDS per wave.
template <int DT, int KIND, class G>
__global__ void __launch_bounds__(64, 2) batch_kernel(BatchArgs A)
{
    __shared__ __attribute__((aligned(16))) unsigned char lds[64 * 288];
    const int lane = threadIdx.x;
    // wave items: the lane's A^(lane * L), L = kBatchLaneBytes of values, held
    // for the whole launch when every item is a wave item, else loaded per
    // wave item (a row item's writer needs those registers)
    constexpr int kt = lane_table(kBatchLaneBytes / Elem<DT>::size);
    const uint32_t *mt = A.lane_tab + (kt * 64 + lane) * 18;
    uint32_t m[18];
    if constexpr (KIND == kKindWave) {
#pragma unroll
        for (int i = 0; i < 18; ++i) m[i] = mt[i];
    }
    if (A.t_start && lane == 0) atomicMin(A.t_start, (unsigned long long)wall_clock64());
    uint64_t next = blockIdx.x;  // static schedule: blockIdx.x + t * gridDim.x
    // dynamic schedule: a wave claims its next item as it starts the current
    // one, so that the claim's round trip overlaps the item's own loads
    uint64_t claim = 0;
    if (A.dynamic && lane == 0) claim = atomicAdd(A.counter, 1ull);
    // a row item's 64-stream blocks [blk, blk_end) still to write: one block
    // per turn of the loop, a new item claimed when none is left
    uint32_t r = 0;
    uint64_t local = 0, blk = 0, blk_end = 0;
    for (;;) {
        if (blk == blk_end) {
            uint64_t item;
            if (A.dynamic) {
                item = lane0_uniform(claim);
                if (item < A.total_items && lane == 0) claim = atomicAdd(A.counter, 1ull);
            } else {
                item = next;
                next += gridDim.x;
            }
            if (item >= A.total_items) break;
            r = find_req(A.prefix, A.nreq, item, lane);
            local = item - A.prefix[r];
            blk = blk_end = 0;
            if constexpr (KIND == kKindRows) {
                const BatchReq &Q = A.reqs[r];
                if (is_row(Q)) {
                    const uint64_t nb = (Q.k + 63) / 64;
                    blk = local * Q.spi;
                    blk_end = blk + Q.spi < nb ? blk + Q.spi : nb;
                }
            }
        }
        const BatchReq R = A.reqs[r];
        if (blk < blk_end) {
            if (R.dtype == 0) row_block<0, G>(R, blk * 64, lds, lane, A);
            else if (R.dtype == 1) row_block<1, G>(R, blk * 64, lds, lane, A);
            else row_block<2, G>(R, blk * 64, lds, lane, A);
            if (++blk < blk_end) continue;
        } else if constexpr (KIND == kKindWave) {
            wave_item<DT, G>(R, local, lds, lane, m, A);
        } else {
            uint32_t mi[18];
#pragma unroll
            for (int i = 0; i < 18; ++i) mi[i] = mt[i];
            wave_item<DT, G>(R, local, lds, lane, mi, A);
        }
        // the item's end (no value returned: no round trip)
        if (A.req_done && lane == 0) atomicMax(&A.req_done[r], (unsigned long long)wall_clock64());
    }
}

__global__ void __launch_bounds__(256) batch_stamp_reset_kernel(unsigned long long *req_done,
                                                                uint64_t n,
                                                                unsigned long long *t_start)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) req_done[i] = 0ull;
    if (i == 0) *t_start = ~0ull;
}

// Entry e with cb_prefix[e] <= s < cb_prefix[e+1] (per-thread binary search).
__device__ __forceinline__ uint32_t cb_entry(const uint64_t *__restrict__ prefix, uint32_t n,
                                             uint64_t s)
{
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (prefix[mid] <= s) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Move the end states of multi-segment streams from scratch to the planes.
// Copy-back slot s belongs to entry e with cb_prefix[e] <= s < cb_prefix[e+1];
// it is stream cb_stream0[e] + (s - cb_prefix[e]) and scratch slot
// cb_scratch0[e] + (s - cb_prefix[e]).
__global__ void __launch_bounds__(256) batch_copyback_kernel(BatchArgs A)
{
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= A.cb_slots) return;
    const uint32_t e = cb_entry(A.cb_prefix, A.n_cb, s);
    const uint64_t off = s - A.cb_prefix[e];
    uint32_t w[6];
    load_state(A.scratch, A.scratch_stride, A.cb_scratch0[e] + off, w);
    store_state(A.planes, A.plane_stride, A.cb_stream0[e] + off, w);
}

template <class G>
static void launch_group_g(const BatchArgs &A, int dtype, int kind, unsigned grid, hipStream_t st)
{
    const dim3 g(grid), b(64);
    if (kind == kKindWave) {
        if (dtype == 0) hipLaunchKernelGGL((batch_kernel<0, kKindWave, G>), g, b, 0, st, A);
        else if (dtype == 1) hipLaunchKernelGGL((batch_kernel<1, kKindWave, G>), g, b, 0, st, A);
        else hipLaunchKernelGGL((batch_kernel<2, kKindWave, G>), g, b, 0, st, A);
    } else {
        if (dtype == 0) hipLaunchKernelGGL((batch_kernel<0, kKindRows, G>), g, b, 0, st, A);
        else if (dtype == 1) hipLaunchKernelGGL((batch_kernel<1, kKindRows, G>), g, b, 0, st, A);
        else hipLaunchKernelGGL((batch_kernel<2, kKindRows, G>), g, b, 0, st, A);
    }
}

hipError_t launch_batch_group(const BatchArgs &A, int dtype, int kind, unsigned grid, int engine,
                              hipStream_t st)
{
    if (A.dynamic) hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(1), 0, st, A.counter);
    if (engine == 1) launch_group_g<GenF>(A, dtype, kind, grid, st);
    else launch_group_g<GenI>(A, dtype, kind, grid, st);
    return hipGetLastError();
}

hipError_t launch_stamp_reset(unsigned long long *req_done, uint64_t n, unsigned long long *t_start,
                              hipStream_t st)
{
    const uint64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(batch_stamp_reset_kernel, dim3((unsigned)(blocks ? blocks : 1)), dim3(256), 0,
                       st, req_done, n, t_start);
    return hipGetLastError();
}

hipError_t launch_copyback(const BatchArgs &A, hipStream_t st)
{
    if (A.cb_slots)
        hipLaunchKernelGGL(batch_copyback_kernel, dim3((unsigned)((A.cb_slots + 255) / 256)),
                           dim3(256), 0, st, A);
    return hipGetLastError();
}

}  // namespace mrg
