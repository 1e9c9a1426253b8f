// Batched generation that allocates nothing: the same plan and persistent
// kernels as mrg_batch_create + mrg_batch_run, with every device buffer the
// run needs (request descriptors, item prefixes, the copy-back table, the
// claim counters and the staged end states of multi-segment streams) carved
// out of one fixed device array, for callers that cannot call hipMalloc.
//
// The array lives for the life of the process on every device the library
// runs on, each device holding its own copy at its own address.  Host code
// never uses the array's name as an address (on the host it is only a
// stand-in for the symbol): the device address comes from
// hipGetSymbolAddress, once per device, and that pointer is what the copies
// and the kernels receive.
#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "batch.h"
#include "internal.h"

using mrg::hip_error;
using mrg::set_error;

namespace {

static __device__ __align__(256) unsigned char scratch[MRG_NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
std::map<int, unsigned char *> g_scratch;  // device -> address of its copy of `scratch`

// Device address of `scratch` on device dev (the current device), looked up
// on the first call for that device.
mrg_status scratch_on(int dev, unsigned char **out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_scratch.find(dev);
    if (it != g_scratch.end()) {
        *out = it->second;
        return MRG_OK;
    }
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol,
                         "hipGetSymbolAddress(batch scratch array)");
    }
    g_scratch.emplace(dev, (unsigned char *)p);
    *out = (unsigned char *)p;
    return MRG_OK;
}

uint64_t align256(uint64_t x) { return (x + 255) & ~(uint64_t)255; }

}  // namespace

extern "C" {

mrg_status mrg_batch_run_noalloc(mrg_streamset ss, const mrg_request *reqs, uint64_t n_reqs,
                                 const mrg_batch_config *cfg, void *stream)
{
    mrg_status st = mrg::check_streamset(ss);
    if (st) return st;
    if (ss->gen != mrg::kGenMRG) return set_error(MRG_EINVAL, "batches take MRG32k3a stream sets only");
    if (n_reqs && !reqs) return set_error(MRG_EINVAL, "null request array");
    if (n_reqs >= ((uint64_t)1 << 31)) return set_error(MRG_ERANGE, "too many requests");
    if ((st = mrg::validate_batch(ss, reqs, n_reqs))) return st;
    const mrg_batch_config c = mrg::batch_config(cfg);
    mrg::HostPlan P;
    mrg::plan_batch(reqs, n_reqs, c, &P);
    if (!P.plan.total_items) return MRG_OK;

    // layout of the array: descriptors | item prefixes | copy-back table
    // (prefix, first streams, first slots) | one claim counter per group |
    // staged end states [6][scratch_slots]
    const uint64_t ncb = P.cb_stream0.size();
    const uint64_t o_prefix = align256(P.plan.reqs.size() * sizeof(mrg::BatchReq));
    const uint64_t o_cb = align256(o_prefix + P.plan.prefix.size() * sizeof(uint64_t));
    const uint64_t o_cnt = align256(o_cb + (3 * ncb + 1) * sizeof(uint64_t));
    const uint64_t o_states = align256(o_cnt + 6 * sizeof(unsigned long long));
    const uint64_t need = o_states + 6 * P.scratch_slots * sizeof(uint32_t);
    if (need > (uint64_t)MRG_NOALLOC_SCRATCH_BYTES)
        return set_error(MRG_ERANGE, "the batch needs %llu bytes of device scratch (%llu requests, "
                         "%llu staged end states); the fixed array holds %llu",
                         (unsigned long long)need, (unsigned long long)P.plan.reqs.size(),
                         (unsigned long long)P.scratch_slots,
                         (unsigned long long)MRG_NOALLOC_SCRATCH_BYTES);

    mrg::DeviceTables tabs;
    if ((st = mrg::device_tables(ss->device, &tabs))) return st;
    unsigned char *d = nullptr;
    if ((st = scratch_on(ss->device, &d))) return st;

    // the host image of everything before the counters (the counters are
    // zeroed by the kernels' own reset launches, the states written by the
    // persistent kernels)
    std::vector<unsigned char> img(o_cnt, 0);
    std::memcpy(img.data(), P.plan.reqs.data(), P.plan.reqs.size() * sizeof(mrg::BatchReq));
    std::memcpy(img.data() + o_prefix, P.plan.prefix.data(), P.plan.prefix.size() * sizeof(uint64_t));
    uint64_t *cb = (uint64_t *)(img.data() + o_cb);
    std::memcpy(cb, P.cb_prefix.data(), (ncb + 1) * sizeof(uint64_t));
    if (ncb) {
        std::memcpy(cb + ncb + 1, P.cb_stream0.data(), ncb * sizeof(uint64_t));
        std::memcpy(cb + 2 * ncb + 1, P.cb_scratch0.data(), ncb * sizeof(uint64_t));
    }

    hipStream_t s = (hipStream_t)stream;
    // every call on this device shares the array: let the earlier work on
    // this stream (a previous call's kernels) finish with it, then upload and
    // wait for the copy, which reads pageable host memory
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipMemcpyAsync(d, img.data(), o_cnt, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_error(e, "batch plan upload to the scratch array");

    mrg::BatchArgs A = {};
    A.dynamic = c.schedule == MRG_SCHEDULE_STATIC ? 0u : 1u;
    A.planes = ss->d_planes;
    A.plane_stride = ss->n;
    A.scratch = (uint32_t *)(d + o_states);
    A.scratch_stride = P.scratch_slots;
    A.table = tabs.table;
    A.lane_tab = tabs.lane_tab;
    A.cb_prefix = (const uint64_t *)(d + o_cb);
    A.cb_stream0 = A.cb_prefix + (ncb + 1);
    A.cb_scratch0 = A.cb_prefix + (2 * ncb + 1);
    A.n_cb = (uint32_t)ncb;
    A.cb_slots = P.cb_prefix.back();
    A.req_done = A.t_start = nullptr;  // no completion stamps
    const uint64_t grid_cap = (uint64_t)tabs.cus * c.waves_per_cu;
    e = mrg::launch_grouped(P.plan, (const mrg::BatchReq *)d, (const uint64_t *)(d + o_prefix),
                            (unsigned long long *)(d + o_cnt), A, grid_cap,
                            mrg::current_tuning().engine, s);
    if (e == hipSuccess) e = mrg::launch_copyback(A, s);
    return e == hipSuccess ? MRG_OK : hip_error(e, "batch kernel launch");
}

}  // extern "C"
