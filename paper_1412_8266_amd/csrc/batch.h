// Device descriptors of the persistent batch kernel (shared by batch.hip and
// the host planner in batch_host.cpp).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace mrg {

constexpr uint32_t kReqSubstreams = 1u;  // streams are substreams of one stream; no write-back
constexpr uint32_t kReqWriteBack = 2u;   // store each stream's end state

// One request as the kernel sees it.  seg > 0: wave items, one per segment of
// seg values of one stream (segs per stream); seg == 0: row items of up to 64
// streams.
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
    uint32_t vec_ok;     // 16-byte stores allowed (aligned rows)
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
    const uint32_t *lane_tab;    // [3][64][18] A^(l*L), L in kLaneSegs
    const uint64_t *cb_prefix;   // [n_cb + 1] copy-back slot prefix
    const uint64_t *cb_stream0;  // [n_cb] plane index of the entry's first stream
    const uint64_t *cb_scratch0; // [n_cb] scratch slot of the entry's first stream
    uint32_t n_cb;
    uint32_t pad;
    uint64_t cb_slots;
};

hipError_t launch_batch(const BatchArgs &A, unsigned grid, int engine, hipStream_t st);

}  // namespace mrg
