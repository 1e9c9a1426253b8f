// C ABI of the TinyMT32 stream sets (sec. 4.2): the parameter search, the
// creation of a set (parameter records checked and built on the device,
// sub-stream starts placed by polynomial jumps) and its description for user
// kernels.  Fills, jumps and state access go through the generic entry
// points in host.cpp, which dispatch on the set's generator.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "internal.h"
#include "tinymt_arith.hpp"

using mrg::hip_error;
using mrg::set_error;

namespace {

constexpr uint64_t kMaxSets = (uint64_t)1 << 20;  // parameter sets per stream set / search
constexpr uint64_t kMaxCandidates = (uint64_t)1 << 31;

// Device buffer freed at scope exit.
struct DevBuf {
    void *p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
    mrg_status alloc(size_t bytes, const char *what)
    {
        hipError_t e = hipMalloc(&p, bytes ? bytes : 4);
        if (e != hipSuccess) {
            p = nullptr;
            return set_error(MRG_ENOMEM, "hipMalloc(%s, %llu bytes): %s", what,
                             (unsigned long long)bytes, hipGetErrorString(e));
        }
        return MRG_OK;
    }
};

// Parameter sets 0 .. count-1 of the search under `master` (the accepted
// candidates in candidate order), testing candidates on the device in
// batches.  Synchronous on `st`.
mrg_status search(uint64_t master, uint64_t count, uint32_t *params, uint64_t *cand,
                  hipStream_t st)
{
    // about 1 in 127 * 2 candidates is kept: batches of ~200 per set wanted,
    // 4 Ki .. 1 Mi candidates
    uint64_t batch = std::min<uint64_t>(std::max<uint64_t>(count * 256, 4096), (uint64_t)1 << 20);
    DevBuf d_flags;
    mrg_status s = d_flags.alloc(batch * 4, "search flags");
    if (s) return s;
    std::vector<uint32_t> flags(batch);
    uint64_t found = 0;
    for (uint64_t c0 = 0; found < count; c0 += batch) {
        if (c0 >= ((uint64_t)1 << 62))
            return set_error(MRG_ERANGE, "parameter search ran past 2^62 candidates");
        hipError_t e = mrg::launch_tmt_candidates(master, c0, batch, (uint32_t *)d_flags.p,
                                                  nullptr, st);
        if (e != hipSuccess) return hip_error(e, "candidate kernel launch");
        e = hipMemcpyAsync(flags.data(), d_flags.p, batch * 4, hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) return hip_error(e, "hipMemcpyAsync(search flags)");
        e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_error(e, "parameter search");
        for (uint64_t i = 0; i < batch && found < count; ++i) {
            if (!((flags[i] >> 16) & 1u)) continue;
            mrg::tmt::candidate(master, c0 + i, params + 3 * found);
            if (cand) cand[found] = c0 + i;
            ++found;
        }
    }
    return MRG_OK;
}

}  // namespace

extern "C" {

mrg_status mrg_tinymt_test_candidates(uint64_t master_seed, uint64_t c0, uint64_t n,
                                      uint32_t *d_flags, uint32_t *d_phi, void *stream)
{
    if (n == 0) return MRG_OK;
    if (!d_flags) return set_error(MRG_EINVAL, "null flag array");
    if (n > kMaxCandidates) return set_error(MRG_ERANGE, "at most 2^31 candidates per call");
    if (c0 > UINT64_MAX - n) return set_error(MRG_ERANGE, "candidate numbers overflow 64 bits");
    int dev;
    mrg_status st = mrg::current_device_id(&dev);
    if (st) return st;
    if ((st = mrg::check_device_span(d_flags, 4 * n, dev, "flag array"))) return st;
    if (d_phi && (st = mrg::check_device_span(d_phi, 16 * n, dev, "polynomial array"))) return st;
    hipError_t e = mrg::launch_tmt_candidates(master_seed, c0, n, d_flags, d_phi,
                                              (hipStream_t)stream);
    return e == hipSuccess ? MRG_OK : hip_error(e, "candidate kernel launch");
}

mrg_status mrg_tinymt_search(uint64_t master_seed, uint64_t count, uint32_t *h_params,
                             uint64_t *h_cand, void *stream)
{
    if (count == 0) return MRG_OK;
    if (!h_params) return set_error(MRG_EINVAL, "null parameter output");
    if (count > kMaxSets) return set_error(MRG_ERANGE, "at most 2^20 parameter sets per search");
    int dev;
    mrg_status st = mrg::current_device_id(&dev);
    if (st) return st;
    return search(master_seed, count, h_params, h_cand, (hipStream_t)stream);
}

mrg_status mrg_streamset_create_tinymt(mrg_streamset *out, uint64_t n_streams,
                                       uint64_t first_stream, uint64_t per_param,
                                       uint64_t master_seed, const uint32_t *h_params,
                                       uint64_t params_first, uint64_t n_params, void *stream)
{
    if (!out) return set_error(MRG_EINVAL, "null argument");
    *out = nullptr;
    if (n_streams == 0) return set_error(MRG_ERANGE, "n_streams must be >= 1");
    if (n_streams - 1 > UINT64_MAX - first_stream)
        return set_error(MRG_ERANGE, "first_stream + n_streams exceeds 2^64");
    if (n_streams > ((uint64_t)1 << 36)) return set_error(MRG_ERANGE, "n_streams above the limit 2^36");
    if (per_param == 0) return set_error(MRG_EINVAL, "per_param must be >= 1");
    const uint64_t q0 = first_stream / per_param;
    const uint64_t qlast = (first_stream + (n_streams - 1)) / per_param;
    const uint64_t nsets = qlast - q0 + 1;
    if (nsets > kMaxSets)
        return set_error(MRG_ERANGE, "%llu parameter sets; at most 2^20 per stream set",
                         (unsigned long long)nsets);
    if (qlast > 0xFFFFFFFFull)
        return set_error(MRG_ERANGE, "parameter set index %llu does not fit the state word",
                         (unsigned long long)qlast);
    hipStream_t st = (hipStream_t)stream;
    std::vector<uint32_t> params;
    if (h_params) {
        if (params_first > q0 || n_params < nsets || qlast - params_first >= n_params)
            return set_error(MRG_ERANGE, "parameter sets [%llu, %llu) do not cover the sets "
                             "[%llu, %llu] of the streams", (unsigned long long)params_first,
                             (unsigned long long)(params_first + n_params),
                             (unsigned long long)q0, (unsigned long long)qlast);
        params.assign(h_params + 3 * (q0 - params_first), h_params + 3 * (qlast - params_first + 1));
    } else {
        if (qlast + 1 > kMaxSets)
            return set_error(MRG_ERANGE, "searching %llu parameter sets; give them instead",
                             (unsigned long long)(qlast + 1));
        int dev;
        mrg_status s = mrg::current_device_id(&dev);
        if (s) return s;
        std::vector<uint32_t> all(3 * (qlast + 1));
        if ((s = search(master_seed, qlast + 1, all.data(), nullptr, st))) return s;
        params.assign(all.begin() + 3 * q0, all.end());
    }
    int dev;
    mrg_status s = mrg::current_device_id(&dev);
    if (s) return s;
    // the records, checked on the device
    DevBuf d_params, d_ok;
    if ((s = d_params.alloc(params.size() * 4, "parameter sets"))) return s;
    if ((s = d_ok.alloc(nsets * 4, "parameter checks"))) return s;
    uint32_t *d_records = nullptr;
    hipError_t e = hipMalloc((void **)&d_records, nsets * mrg::tmt::kRecordWords * 4);
    if (e != hipSuccess)
        return set_error(MRG_ENOMEM, "hipMalloc(%llu parameter records): %s",
                         (unsigned long long)nsets, hipGetErrorString(e));
    auto fail = [&](mrg_status r) {
        (void)hipFree(d_records);
        return r;
    };
    e = hipMemcpyAsync(d_params.p, params.data(), params.size() * 4, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return fail(hip_error(e, "hipMemcpyAsync(parameter sets)"));
    e = mrg::launch_tmt_records((const uint32_t *)d_params.p, nsets, d_records, (uint32_t *)d_ok.p, st);
    if (e != hipSuccess) return fail(hip_error(e, "record kernel launch"));
    std::vector<uint32_t> ok(nsets);
    e = hipMemcpyAsync(ok.data(), d_ok.p, nsets * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(hip_error(e, "parameter checks"));
    for (uint64_t i = 0; i < nsets; ++i)
        if (!ok[i])
            return fail(set_error(MRG_EINVAL, "parameter set %llu (%08x %08x %08x) has no "
                                  "irreducible characteristic polynomial of degree 127",
                                  (unsigned long long)(q0 + i), params[3 * i], params[3 * i + 1],
                                  params[3 * i + 2]));
    auto *ss = new (std::nothrow) mrg_streamset_s;
    if (!ss) return fail(set_error(MRG_ENOMEM, "host allocation"));
    ss->device = dev;
    ss->n = n_streams;
    ss->first = first_stream;
    ss->gen = mrg::kGenTinyMT;
    ss->d_records = d_records;
    ss->per_param = per_param;
    ss->q0 = q0;
    ss->n_sets = nsets;
    e = hipMalloc(&ss->d_planes, 6 * n_streams * sizeof(uint32_t));
    if (e != hipSuccess) {
        delete ss;
        return fail(set_error(MRG_ENOMEM, "hipMalloc(%llu states): %s",
                              (unsigned long long)n_streams, hipGetErrorString(e)));
    }
    e = mrg::launch_tmt_init(ss->d_planes, n_streams, n_streams, first_stream, per_param, q0,
                             master_seed, d_records, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);  // before the parameter buffers go
    if (e != hipSuccess) {
        (void)hipFree(ss->d_planes);
        delete ss;
        return fail(hip_error(e, "tinymt init kernel"));
    }
    *out = ss;
    return MRG_OK;
}

mrg_status mrg_streamset_tinymt_info(mrg_streamset ss, uint64_t *per_param, uint64_t *q0,
                                     uint64_t *n_sets, const void **d_records)
{
    if (!ss) return set_error(MRG_EINVAL, "null stream set");
    if (ss->gen != mrg::kGenTinyMT) return set_error(MRG_EINVAL, "not a TinyMT32 stream set");
    if (per_param) *per_param = ss->per_param;
    if (q0) *q0 = ss->q0;
    if (n_sets) *n_sets = ss->n_sets;
    if (d_records) *d_records = ss->d_records;
    return MRG_OK;
}

}  // extern "C"
