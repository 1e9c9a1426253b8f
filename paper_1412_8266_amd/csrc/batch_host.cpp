// Batched generation: planner, hipGraph capture, per-request baseline and the
// autotuner of the persistent batch kernel (batch.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "batch.h"
#include "internal.h"

using mrg::hip_error;
using mrg::set_error;

struct mrg_batch_s {
    mrg_streamset ss = nullptr;
    int device = -1;
    std::vector<mrg_request> reqs;   // as given (zero-size ones included)
    mrg_batch_config cfg = {};       // effective configuration
    mrg::DeviceTables tabs;
    int engine = 1;

    // plan (host mirror and device copies)
    std::vector<mrg::BatchReq> breqs;
    std::vector<uint64_t> prefix;    // [nreq + 1]
    std::vector<uint64_t> cb_prefix, cb_stream0, cb_scratch0;
    uint64_t total_items = 0, scratch_slots = 0, samples = 0, bytes = 0;
    mrg::BatchReq *d_reqs = nullptr;
    uint64_t *d_prefix = nullptr;
    uint64_t *d_solo = nullptr;      // [nreq][2]: {0, items of request r}
    uint64_t *d_cb = nullptr;        // cb_prefix | cb_stream0 | cb_scratch0
    unsigned long long *d_counter = nullptr;
    uint32_t *d_scratch = nullptr;
    unsigned grid = 0;

    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

void free_plan(mrg_batch b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    for (void *p : {(void *)b->d_reqs, (void *)b->d_prefix, (void *)b->d_solo, (void *)b->d_cb,
                    (void *)b->d_counter, (void *)b->d_scratch})
        if (p) (void)hipFree(p);
    b->d_reqs = nullptr;
    b->d_prefix = b->d_solo = b->d_cb = nullptr;
    b->d_counter = nullptr;
    b->d_scratch = nullptr;
}

mrg_batch_config effective(const mrg_batch_config *c)
{
    mrg_batch_config e = {};
    if (c) e = *c;
    if (!e.segment_bytes) e.segment_bytes = 256 * 1024;
    if (!e.waves_per_cu) e.waves_per_cu = 16;
    if (!e.wave_min_bytes) e.wave_min_bytes = 16 * 1024;
    if (e.schedule != MRG_SCHEDULE_STATIC) e.schedule = MRG_SCHEDULE_DYNAMIC;
    return e;
}

template <class T>
mrg_status upload(T **dst, const std::vector<T> &src, const char *what)
{
    const size_t bytes = std::max<size_t>(src.size(), 1) * sizeof(T);
    hipError_t e = hipMalloc((void **)dst, bytes);
    if (e != hipSuccess) return set_error(MRG_ENOMEM, "hipMalloc(%s): %s", what, hipGetErrorString(e));
    if (!src.empty()) {
        e = hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_error(e, what);
    }
    return MRG_OK;
}

// Cut the requests into work items under b->cfg and upload the plan.
mrg_status build_plan(mrg_batch b)
{
    free_plan(b);
    b->breqs.clear();
    b->prefix.assign(1, 0);
    b->cb_prefix.assign(1, 0);
    b->cb_stream0.clear();
    b->cb_scratch0.clear();
    b->total_items = b->scratch_slots = b->samples = b->bytes = 0;
    std::vector<uint64_t> solo;
    for (const mrg_request &q : b->reqs) {
        if (!q.count || !q.n_per_stream) continue;
        const uint64_t es = q.dtype == MRG_F64 ? 8 : 4;
        const uint64_t chunk = 64 * (256 / es);  // values per wave_fill chunk
        mrg::BatchReq R = {};
        R.out = (unsigned char *)q.d_out;
        R.stream0 = q.first;
        R.k = q.count;
        R.n = q.n_per_stream;
        R.sub0 = q.substream0;
        R.dtype = (uint32_t)q.dtype;
        R.flags = (q.flags & MRG_REQ_SUBSTREAMS) ? mrg::kReqSubstreams : mrg::kReqWriteBack;
        R.vec_ok = ((uintptr_t)q.d_out % 16 == 0) && ((R.n * es) % 16 == 0);
        uint64_t items;
        if (R.n * es >= b->cfg.wave_min_bytes) {
            uint64_t seg = b->cfg.segment_bytes / es / chunk * chunk;
            if (seg < chunk) seg = chunk;
            R.seg = seg;
            R.segs = (R.n + seg - 1) / seg;
            items = R.k * R.segs;
            if (R.segs > 1 && (R.flags & mrg::kReqWriteBack)) {
                R.scratch0 = b->scratch_slots;
                b->cb_stream0.push_back(R.stream0);
                b->cb_scratch0.push_back(R.scratch0);
                b->cb_prefix.push_back(b->cb_prefix.back() + R.k);
                b->scratch_slots += R.k;
            }
        } else {
            R.seg = 0;
            R.segs = 1;
            items = (R.k + 63) / 64;
        }
        b->breqs.push_back(R);
        solo.push_back(0);
        solo.push_back(items);
        b->total_items += items;
        b->prefix.push_back(b->total_items);
        b->samples += R.k * R.n;
        b->bytes += R.k * R.n * es;
    }
    mrg_status st;
    if ((st = upload(&b->d_reqs, b->breqs, "batch requests"))) return st;
    if ((st = upload(&b->d_prefix, b->prefix, "batch prefix"))) return st;
    if ((st = upload(&b->d_solo, solo, "batch solo prefix"))) return st;
    std::vector<uint64_t> cb(b->cb_prefix);
    cb.insert(cb.end(), b->cb_stream0.begin(), b->cb_stream0.end());
    cb.insert(cb.end(), b->cb_scratch0.begin(), b->cb_scratch0.end());
    if ((st = upload(&b->d_cb, cb, "batch copy-back"))) return st;
    hipError_t e = hipMalloc((void **)&b->d_counter, sizeof(unsigned long long));
    if (e != hipSuccess) return set_error(MRG_ENOMEM, "hipMalloc(counter)");
    if (b->scratch_slots) {
        e = hipMalloc((void **)&b->d_scratch, 6 * b->scratch_slots * sizeof(uint32_t));
        if (e != hipSuccess)
            return set_error(MRG_ENOMEM, "hipMalloc(batch scratch, %llu states)",
                             (unsigned long long)b->scratch_slots);
    }
    const uint64_t cap = (uint64_t)b->tabs.cus * b->cfg.waves_per_cu;
    b->grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(cap, b->total_items));
    return MRG_OK;
}

mrg::BatchArgs args_of(mrg_batch b)
{
    mrg::BatchArgs A = {};
    A.reqs = b->d_reqs;
    A.prefix = b->d_prefix;
    A.nreq = (uint32_t)b->breqs.size();
    A.dynamic = b->cfg.schedule == MRG_SCHEDULE_STATIC ? 0u : 1u;
    A.total_items = b->total_items;
    A.counter = b->d_counter;
    A.planes = b->ss->d_planes;
    A.plane_stride = b->ss->n;
    A.scratch = b->d_scratch;
    A.scratch_stride = b->scratch_slots;
    A.table = b->tabs.table;
    A.lane_tab = b->tabs.lane_tab;
    const uint32_t ncb = (uint32_t)b->cb_stream0.size();
    A.cb_prefix = b->d_cb;
    A.cb_stream0 = b->d_cb + (ncb + 1);
    A.cb_scratch0 = b->d_cb + (ncb + 1) + ncb;
    A.n_cb = ncb;
    A.cb_slots = b->cb_prefix.back();
    return A;
}

mrg_status capture(mrg_batch b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    if (!b->total_items) return MRG_OK;
    hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_error(e, "hipStreamBeginCapture");
    hipError_t le = mrg::launch_batch(args_of(b), b->grid, b->engine, b->cap_stream);
    e = hipStreamEndCapture(b->cap_stream, &b->graph);
    if (le != hipSuccess) return hip_error(le, "batch kernel capture");
    if (e != hipSuccess) return hip_error(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_error(e, "hipGraphInstantiate");
    return MRG_OK;
}

mrg_status validate(mrg_streamset ss, const mrg_request *reqs, uint64_t n)
{
    std::vector<std::pair<uint64_t, uint64_t>> spans;
    for (uint64_t i = 0; i < n; ++i) {
        const mrg_request &q = reqs[i];
        if (q.dtype != MRG_U32 && q.dtype != MRG_F32 && q.dtype != MRG_F64)
            return set_error(MRG_EINVAL, "request %llu: unknown dtype %d", (unsigned long long)i,
                             (int)q.dtype);
        if (q.flags & ~(uint32_t)MRG_REQ_SUBSTREAMS)
            return set_error(MRG_EINVAL, "request %llu: unknown flags", (unsigned long long)i);
        if (!q.count || !q.n_per_stream) continue;
        const uint64_t es = q.dtype == MRG_F64 ? 8 : 4;
        if (!q.d_out || (uintptr_t)q.d_out % es)
            return set_error(MRG_EINVAL, "request %llu: null or misaligned output",
                             (unsigned long long)i);
        if (q.n_per_stream > UINT64_MAX / es / q.count)
            return set_error(MRG_ERANGE, "request %llu: output size overflows", (unsigned long long)i);
        if (q.flags & MRG_REQ_SUBSTREAMS) {
            if (q.first >= ss->n)
                return set_error(MRG_ERANGE, "request %llu: stream outside the set", (unsigned long long)i);
            if (q.count - 1 > ((uint64_t)1 << 62) - q.substream0)
                return set_error(MRG_ERANGE, "request %llu: substream index overflow",
                                 (unsigned long long)i);
        } else {
            if (q.first > ss->n || q.count > ss->n - q.first)
                return set_error(MRG_ERANGE, "request %llu: streams outside the set",
                                 (unsigned long long)i);
            spans.emplace_back(q.first, q.first + q.count);
        }
    }
    std::sort(spans.begin(), spans.end());
    for (size_t i = 1; i < spans.size(); ++i)
        if (spans[i].first < spans[i - 1].second)
            return set_error(MRG_EINVAL, "requests overlap on streams [%llu, %llu)",
                             (unsigned long long)spans[i].first,
                             (unsigned long long)std::min(spans[i].second, spans[i - 1].second));
    return MRG_OK;
}

}  // namespace

extern "C" {

mrg_status mrg_batch_create(mrg_batch *out, mrg_streamset ss, const mrg_request *reqs,
                            uint64_t n_reqs, const mrg_batch_config *cfg)
{
    if (!out) return set_error(MRG_EINVAL, "null output handle");
    *out = nullptr;
    mrg_status st = mrg::check_streamset(ss);
    if (st) return st;
    if (n_reqs && !reqs) return set_error(MRG_EINVAL, "null request array");
    if (n_reqs >= ((uint64_t)1 << 31)) return set_error(MRG_ERANGE, "too many requests");
    if ((st = validate(ss, reqs, n_reqs))) return st;
    auto *b = new (std::nothrow) mrg_batch_s;
    if (!b) return set_error(MRG_ENOMEM, "host allocation");
    b->ss = ss;
    b->device = ss->device;
    b->reqs.assign(reqs, reqs + n_reqs);
    b->cfg = effective(cfg);
    b->engine = mrg::current_tuning().engine;
    if ((st = mrg::device_tables(ss->device, &b->tabs))) {
        delete b;
        return st;
    }
    hipError_t e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete b;
        return hip_error(e, "hipStreamCreate");
    }
    if ((st = build_plan(b)) || (st = capture(b))) {
        mrg_batch_destroy(b);
        return st;
    }
    *out = b;
    return MRG_OK;
}

mrg_status mrg_batch_destroy(mrg_batch b)
{
    if (!b) return MRG_OK;
    (void)hipDeviceSynchronize();
    free_plan(b);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    delete b;
    return MRG_OK;
}

mrg_status mrg_batch_run(mrg_batch b, void *stream)
{
    if (!b) return set_error(MRG_EINVAL, "null batch");
    if (!b->exec) return MRG_OK;
    hipError_t e = hipGraphLaunch(b->exec, (hipStream_t)stream);
    return e == hipSuccess ? MRG_OK : hip_error(e, "hipGraphLaunch");
}

mrg_status mrg_batch_run_direct(mrg_batch b, void *stream)
{
    if (!b) return set_error(MRG_EINVAL, "null batch");
    if (!b->total_items) return MRG_OK;
    hipError_t e = mrg::launch_batch(args_of(b), b->grid, b->engine, (hipStream_t)stream);
    return e == hipSuccess ? MRG_OK : hip_error(e, "batch kernel launch");
}

mrg_status mrg_batch_run_per_request(mrg_batch b, void *stream)
{
    if (!b) return set_error(MRG_EINVAL, "null batch");
    size_t r = 0;
    for (const mrg_request &q : b->reqs) {
        if (!q.count || !q.n_per_stream) continue;
        mrg_status st;
        if (q.flags & MRG_REQ_SUBSTREAMS) {
            // the batch kernel on this one request
            mrg::BatchArgs A = args_of(b);
            A.reqs = b->d_reqs + r;
            A.prefix = b->d_solo + 2 * r;
            A.nreq = 1;
            A.total_items = b->prefix[r + 1] - b->prefix[r];
            A.n_cb = 0;
            A.cb_slots = 0;
            const uint64_t cap = (uint64_t)b->tabs.cus * b->cfg.waves_per_cu;
            const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min(cap, A.total_items));
            hipError_t e = mrg::launch_batch(A, grid, b->engine, (hipStream_t)stream);
            st = e == hipSuccess ? MRG_OK : hip_error(e, "batch kernel launch");
        } else {
            st = mrg_fill(b->ss, q.first, q.count, q.n_per_stream, (mrg_dtype)q.dtype,
                          MRG_STREAM_MAJOR, q.d_out, stream);
        }
        if (st) return st;
        ++r;
    }
    return MRG_OK;
}

mrg_status mrg_batch_info(mrg_batch b, mrg_batch_info_t *info)
{
    if (!b || !info) return set_error(MRG_EINVAL, "null argument");
    info->requests = b->breqs.size();
    info->items = b->total_items;
    info->samples = b->samples;
    info->bytes = b->bytes;
    info->grid = b->grid;
    info->scratch_states = b->scratch_slots;
    info->config = b->cfg;
    return MRG_OK;
}

mrg_status mrg_batch_autotune(mrg_batch b, const mrg_batch_config *cands, uint32_t n_cands,
                              uint32_t reps, void *stream, uint32_t *best_out, float *ms_out)
{
    if (!b || !cands || !n_cands) return set_error(MRG_EINVAL, "null argument or no candidates");
    if (!reps) reps = 1;
    hipStream_t st = (hipStream_t)stream;
    // the runs advance the streams: save the states and restore them after
    const size_t plane_bytes = 6 * b->ss->n * sizeof(uint32_t);
    void *saved = nullptr;
    hipError_t e = hipMalloc(&saved, plane_bytes);
    if (e != hipSuccess) return set_error(MRG_ENOMEM, "hipMalloc(state backup)");
    e = hipMemcpyAsync(saved, b->ss->d_planes, plane_bytes, hipMemcpyDeviceToDevice, st);
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    mrg_status status = e == hipSuccess ? MRG_OK : hip_error(e, "autotune setup");
    uint32_t best = 0;
    float best_ms = 0;
    const mrg_batch_config keep = b->cfg;
    for (uint32_t i = 0; i < n_cands && status == MRG_OK; ++i) {
        b->cfg = effective(&cands[i]);
        if ((status = build_plan(b)) || (status = capture(b))) break;
        if ((status = mrg_batch_run(b, stream))) break;  // warm-up
        (void)hipEventRecord(t0, st);
        for (uint32_t r = 0; r < reps && status == MRG_OK; ++r) status = mrg_batch_run(b, stream);
        (void)hipEventRecord(t1, st);
        if (status) break;
        e = hipEventSynchronize(t1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
        if (e != hipSuccess) {
            status = hip_error(e, "autotune timing");
            break;
        }
        ms /= (float)reps;
        if (ms_out) ms_out[i] = ms;
        if (i == 0 || ms < best_ms) {
            best = i;
            best_ms = ms;
        }
    }
    (void)hipStreamSynchronize(st);
    e = hipMemcpyAsync(b->ss->d_planes, saved, plane_bytes, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess && status == MRG_OK) status = hip_error(e, "state restore");
    if (status == MRG_OK) {
        b->cfg = effective(&cands[best]);
        status = build_plan(b);
        if (status == MRG_OK) status = capture(b);
    } else {
        b->cfg = keep;
        if (build_plan(b) == MRG_OK) (void)capture(b);
    }
    (void)hipStreamSynchronize(st);
    (void)hipFree(saved);
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    if (best_out) *best_out = best;
    return status;
}

}  // extern "C"
