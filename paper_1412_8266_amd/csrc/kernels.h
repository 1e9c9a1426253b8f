// Internal interface between the C-ABI host code and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mrg32k3a_device.h"  // table layout (kTableWindows, kTableWindowWords)

namespace mrg {

constexpr int kTableWords = 2 * kTableWindows * kTableWindowWords;

struct InitSeed { uint32_t w[6]; };
struct JumpMatrices { uint32_t m[18]; };  // component 1 then component 2

hipError_t launch_init(uint32_t *planes, uint64_t plane_stride, uint64_t count, uint64_t g0,
                       const InitSeed &seed, const uint32_t *table, int w_lo, int w_hi,
                       hipStream_t st);
hipError_t launch_jump(uint32_t *planes, uint64_t plane_stride, uint64_t first, uint64_t count,
                       const uint64_t *d_exp, const uint32_t *table, hipStream_t st);
hipError_t launch_jump_uniform(uint32_t *planes, uint64_t plane_stride, uint64_t first,
                               uint64_t count, const JumpMatrices &J, hipStream_t st);
// Generation engine (0: integer lazy words, 1: binary64 near-canonical words),
// bytes per row per LDS tile (128 or 256) of the lane-per-stream fill, and
// the stream-major strategy (0: automatic, 1: lane per stream, 2: wave per
// stream).
struct FillTuning {
    int engine = 1;
    int tile_bytes = 0;       // lane per stream: 0 = 128 for rows under 1 KiB, else 256
    int strategy = 0;
    int coop_wgs_per_cu = 0;  // wave per stream: 0 = one workgroup per stream group
    int coop_lanes = 0;       // wave per stream: lanes per stream (64, 32, 16, 8; 0 automatic)
    int coop_order = 0;       // wave per stream: 0 chunked (one front), 1 one range per XCD
};

// Lane tables of the wave-per-stream writer: table lane_table(L) holds
// A^(l*L) for l < 64 and each lane-segment length L = 16, 32, ..., 512 values
// (a chunk's members, and the shorter members of a chunk where rows end);
// table kHeadTable holds A^l (the values before a row's first 128-byte line
// boundary).
constexpr int kNumLaneTabs = 33;
constexpr int kHeadTable = 32;
__host__ __device__ constexpr int lane_table(int L) { return L / 16 - 1; }

// How one stream-major fill is launched (chosen on the host).
struct FillLaunch {
    int kernel = 0;                     // 0 lane per stream, 1 wave per stream
    int L = 0;                          // values per lane per chunk (wave per stream)
    int lanes = 64;                     // lanes per stream (wave per stream)
    const uint32_t *lane_tab = nullptr; // [64][18]: A^(l*L), component 1 then 2 (lane l % lanes)
    const uint32_t *tabs = nullptr;     // all lane tables ([kNumLaneTabs][64][18])
    const uint32_t *table = nullptr;    // windowed jump tables (end state of a partial chunk)
    unsigned grid = 0;                  // workgroups (wave per stream)
    int order = 0;                      // group order (FillTuning::coop_order)
    int whole = 0;                      // rows on 128-byte lines, whole chunks only (fast writer)
};

hipError_t launch_fill(uint32_t *planes, uint64_t plane_stride, uint64_t first, uint64_t count,
                       uint64_t n, int dtype, int layout, void *out,
                       const FillLaunch &fl, const FillTuning &tune, hipStream_t st);

// Random spacing: stream g0 + s of a set starts at the state expanded from
// SplitMix64 output g0 + s of the master seed.
hipError_t launch_random_init(uint32_t *planes, uint64_t plane_stride, uint64_t count,
                              uint64_t g0, uint64_t master, hipStream_t st);

// Leapfrog with each player's cards in a row: P players, K cards each; work
// items of KB = min(K, 64) card columns x T = R*Ts players (R = 64 / KB lanes
// per column), nseg segments per column block, items = column blocks x nseg.
struct LeapArgs {
    uint64_t P = 0, K = 0, T = 0, Ts = 0, nseg = 0, items = 0;
    int KB = 64, R = 1;
    JumpMatrices J63 = {};   // A^(63*P): to the next column block (R = 1)
    JumpMatrices Jseg = {};  // A^(T - Ts): to the next segment (R > 1)
};

// One stream partitioned (chosen on the host): kind 0 writes its outputs
// [0, nfull*B + rem) in order, in blocks of B values (64 lanes per block, L
// values per lane per chunk); kind 1 deals them to players, each player's
// cards in a row.
struct PartitionLaunch {
    int kind = 0;
    int L = 0;
    uint64_t nfull = 0, B = 0, rem = 0;  // kind 0
    LeapArgs leap;                       // kind 1
    const uint32_t *lane_tab = nullptr;  // kind 0: [64][18] A^(l*L)
    const uint32_t *tabs = nullptr;      // kind 0: all lane tables
    const uint32_t *table = nullptr;     // windowed jump tables
    unsigned grid = 0;
};
hipError_t launch_partition(const uint32_t *planes, uint64_t plane_stride, uint64_t sidx,
                            int dtype, const PartitionLaunch &pl, void *out, int engine,
                            hipStream_t st);

// Philox4x32-10 stream sets (philox.hip): states (position, id, key); fills
// leave the positions to a following launch_philox_jump.
hipError_t launch_philox_init(uint32_t *planes, uint64_t plane_stride, uint64_t count,
                              uint64_t g0, uint64_t key, hipStream_t st);
hipError_t launch_philox_jump(uint32_t *planes, uint64_t plane_stride, uint64_t first,
                              uint64_t count, const uint64_t *d_exp, uint64_t e, hipStream_t st);
hipError_t launch_philox_fill(const uint32_t *planes, uint64_t plane_stride, uint64_t first,
                              uint64_t count, uint64_t n, int dtype, int layout, void *out,
                              hipStream_t st);

// TinyMT32 stream sets (tinymt.hip): states (s0, s1, s2, s3, q, 0), one
// record of tmt::kRecordWords words per parameter set (sets q0, q0 + 1, ...).
// Candidates: flags[i] = L | accepted << 16 for candidate c0 + i, phis
// (optional) its characteristic polynomial.  Records: ok[i] = 1 when set i
// is accepted.
hipError_t launch_tmt_candidates(uint64_t master, uint64_t c0, uint64_t n, uint32_t *flags,
                                 uint32_t *phis, hipStream_t st);
hipError_t launch_tmt_records(const uint32_t *params, uint64_t n, uint32_t *records, uint32_t *ok,
                              hipStream_t st);
hipError_t launch_tmt_init(uint32_t *planes, uint64_t plane_stride, uint64_t count, uint64_t g0,
                           uint64_t per_param, uint64_t q0, uint64_t master,
                           const uint32_t *records, hipStream_t st);
hipError_t launch_tmt_jump(uint32_t *planes, uint64_t plane_stride, uint64_t first, uint64_t count,
                           const uint64_t *d_exp, const uint64_t e[3], const uint32_t *records,
                           uint64_t q0, hipStream_t st);
hipError_t launch_tmt_fill(uint32_t *planes, uint64_t plane_stride, uint64_t first, uint64_t count,
                           uint64_t n, int dtype, int layout, void *out, const uint32_t *records,
                           uint64_t q0, int tile_bytes, hipStream_t st);

// Store-only bandwidth probes (probe.hip): pattern 0 streaming, 1 the
// wave-per-stream fill's line geometry.
hipError_t launch_write_probe(void *out, uint64_t bytes, int pattern, hipStream_t st);

}  // namespace mrg
