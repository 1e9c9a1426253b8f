// Descriptors of the persistent batch kernels and the grouping of requests
// into launch groups (shared by batch.hip, the planner in
// batch_host.cpp and the server in serve.cpp).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "kernels.h"
#include "mrg32k3a_gpu.h"

namespace mrg {

constexpr uint32_t kReqSubstreams = 1u;  // streams are substreams of one stream; no write-back
constexpr uint32_t kReqWriteBack = 2u;   // store each stream's end state

// Bytes each lane of a wave item generates per chunk (64 lanes per chunk):
// the lane's start state costs one matrix-vector product per chunk, so longer
// lane segments spend fewer instructions per sample on it.
constexpr int kBatchLaneBytes = 1024;

// Launch kinds.  kKindWave: wave items of one dtype.  kKindRows: the row
// items of every dtype (one lane per stream, up to 64 streams per item),
// largest first, then the wave items of one dtype, in one persistent launch:
// row items are too few and too uneven to fill the chip on their own (a
// stream of up to 16 KiB per lane), and the wave items that follow them fill
// the slots their tail leaves idle.
constexpr int kKindWave = 0;
constexpr int kKindRows = 1;

// One request as the kernel sees it.  seg > 0: wave items, one per segment of
// seg values of one stream (segs per stream), or, when a stream fits one
// segment, one per spi consecutive whole streams; seg == 0: row items of spi
// consecutive blocks of up to 64 streams each.
struct BatchReq {
    unsigned char *out;  // [k, n] stream-major output of dtype elements
    uint64_t stream0;    // plane index of stream 0 (substream mode: of the one stream)
    uint64_t k;          // streams
    uint64_t n;          // values per stream
    uint64_t seg;        // values per wave item (multiple of the chunk), 0 for row items
    uint64_t segs;       // wave items per stream
    uint64_t sub0;       // substream mode: stream j is substream sub0 + j
    uint64_t scratch0;   // first scratch slot (multi-segment write-back)
    uint32_t dtype;      // 0 u32, 1 f32, 2 f64
    uint32_t flags;      // kReqSubstreams | kReqWriteBack
    uint32_t spi;        // wave items: whole streams per item (segs == 1), else 1;
                         // row items: 64-stream blocks per item
    uint32_t pad;
};

struct BatchArgs {
    const BatchReq *reqs;
    const uint64_t *prefix;      // [nreq + 1] first item of each request
    uint32_t nreq;
    uint32_t dynamic;            // 1: atomic counter, 0: round robin
    uint64_t total_items;
    unsigned long long *counter;
    uint32_t *planes;
    uint64_t plane_stride;
    uint32_t *scratch;           // [6][scratch_stride]
    uint64_t scratch_stride;
    const uint32_t *table;       // windowed jump tables
    const uint32_t *lane_tab;    // [kNumLaneSegs][64][18] A^(l*L), L in kLaneSegs
    const uint64_t *cb_prefix;   // [n_cb + 1] copy-back slot prefix
    const uint64_t *cb_stream0;  // [n_cb] plane index of the entry's first stream
    const uint64_t *cb_scratch0; // [n_cb] scratch slot of the entry's first stream
    uint32_t n_cb;
    uint32_t pad;
    uint64_t cb_slots;
    // completion stamps (both NULL: none): per request of the group, the
    // latest wall clock at which one of its items ended (a max over items);
    // the earliest workgroup start of the run
    unsigned long long *req_done;
    unsigned long long *t_start;
};

__host__ __device__ inline bool is_row(const BatchReq &R) { return R.seg == 0; }

// Row items carry blocks of 64 streams until they hold about kRowItemBytes of
// output (at most 16 blocks): an item pays its claim, request lookup and
// descriptor load once, which for rows of a few hundred bytes cost as much as
// writing them.
constexpr uint64_t kRowItemBytes = 128 * 1024;
inline uint32_t row_blocks_per_item(uint64_t n, uint64_t es)
{
    const uint64_t b = kRowItemBytes / (64 * n * es);
    return (uint32_t)(b < 1 ? 1 : b > 16 ? 16 : b);
}

inline uint64_t items_of(const BatchReq &R)
{
    if (!R.seg) return ((R.k + 63) / 64 + R.spi - 1) / R.spi;
    return R.spi > 1 ? (R.k + R.spi - 1) / R.spi : R.k * R.segs;
}

// Requests reordered into launch groups, each with its own item prefix:
// one per dtype with wave items, the first launched (least output) led by the
// row items of every dtype (kKindRows; alone when no request has wave items);
// built on the host, uploaded as one request array and one prefix array.
struct Grouped {
    struct Group {
        int dtype, kind;  // kKindRows: dtype is the wave items' (rows carry their own)
        uint32_t req_off, nreq;  // slice of `reqs`
        uint32_t prefix_off;     // slice of `prefix` (nreq + 1 entries)
        uint64_t items;
    };
    std::vector<BatchReq> reqs;
    std::vector<uint64_t> prefix;
    std::vector<Group> groups;   // non-empty groups, least output first (launch order)
    std::vector<uint32_t> pos;   // input request i -> index in reqs
    uint64_t total_items = 0;
};

void group_requests(const std::vector<BatchReq> &in, Grouped *out);

// A batch cut into work items on the host, before any upload: the grouped
// descriptors, which input request each non-empty one came from, and the
// copy-back table of multi-segment streams (entry e covers copy-back slots
// [cb_prefix[e], cb_prefix[e+1]): streams cb_stream0[e] + j, staged in scratch
// slots cb_scratch0[e] + j).
struct HostPlan {
    std::vector<BatchReq> in;       // non-empty requests in input order
    Grouped plan;
    std::vector<uint32_t> req_of;   // non-empty request -> input index
    std::vector<uint64_t> cb_prefix, cb_stream0, cb_scratch0;
    uint64_t scratch_slots = 0, samples = 0, bytes = 0;
};
// Work items of each request under cfg (an effective configuration).
void plan_batch(const mrg_request *reqs, uint64_t n, const mrg_batch_config &cfg, HostPlan *out);
// cfg with defaults filled in (cfg may be NULL).
mrg_batch_config batch_config(const mrg_batch_config *cfg);
// The checks of mrg_batch_create: dtypes, flags, outputs (device memory of
// the set's device, inside one allocation), stream ranges, overlaps.
mrg_status validate_batch(mrg_streamset ss, const mrg_request *reqs, uint64_t n);

// Launch every group (counter reset + persistent kernel) on one stream.
// base carries the state planes, tables, scratch and schedule; counters holds
// one counter per group.
hipError_t launch_grouped(const Grouped &g, const BatchReq *d_reqs, const uint64_t *d_prefix,
                          unsigned long long *d_counters, const BatchArgs &base,
                          uint64_t grid_cap, int engine, hipStream_t st);

hipError_t launch_batch_group(const BatchArgs &A, int dtype, int kind, unsigned grid, int engine,
                              hipStream_t st);
hipError_t launch_copyback(const BatchArgs &A, hipStream_t st);
// Zero n completion stamps and set the start stamp to its maximum (before a run).
hipError_t launch_stamp_reset(unsigned long long *req_done, uint64_t n, unsigned long long *t_start,
                              hipStream_t st);

}  // namespace mrg
