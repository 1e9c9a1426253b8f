// Library-internal declarations shared by the C-ABI translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"
#include "mrg32k3a_gpu.h"

struct mrg_streamset_s {
    int device = -1;
    uint64_t n = 0;                // streams in the set
    uint64_t first = 0;            // global index of stream 0 of the set
    uint32_t seed[6] = {};         // base state (global stream 0)
    int gen = 0;                   // 0 MRG32k3a, 1 Philox4x32-10, 2 TinyMT32
    uint32_t *d_planes = nullptr;  // [6][n]
    // TinyMT32 sets: records of parameter sets q0 .. q0 + n_sets - 1, each
    // shared by per_param consecutive global streams
    uint32_t *d_records = nullptr;
    uint64_t per_param = 0, q0 = 0, n_sets = 0;
};

namespace mrg {
constexpr int kGenMRG = 0, kGenPhilox = 1, kGenTinyMT = 2;
}

namespace mrg {

// Record the calling thread's error text and return s.
mrg_status set_error(mrg_status s, const char *fmt, ...);
mrg_status hip_error(hipError_t e, const char *what);

// Device-resident tables of one device (created on first use).
struct DeviceTables {
    const uint32_t *table = nullptr;     // windowed jump tables, kTableWords words
    const uint32_t *lane_tab = nullptr;  // [kNumLaneSegs][64][18]
    int cus = 256;
};
mrg_status device_tables(int dev, DeviceTables *out);

FillTuning current_tuning();

// The calling thread's current HIP device (MRG_ENODEV when there is none).
mrg_status current_device_id(int *dev);

// Stream set usable on the current device; range inside the set.
mrg_status check_streamset(mrg_streamset ss);
mrg_status check_range(mrg_streamset ss, uint64_t first, uint64_t count);
// [p, p + bytes) is device memory of device dev (or managed memory) inside
// one allocation, else MRG_EINVAL / MRG_ERANGE naming `what`.  Kernels store
// through such pointers, so a host address must never reach them.
mrg_status check_device_span(const void *p, uint64_t bytes, int dev, const char *what);

}  // namespace mrg
