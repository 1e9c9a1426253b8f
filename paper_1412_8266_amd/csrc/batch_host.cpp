// Batched generation: planner, hipGraph capture, per-request reference
// schedule and the autotuner of the persistent batch kernels (batch.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <iterator>
#include <new>
#include <vector>

#include "batch.h"
#include "internal.h"

using mrg::hip_error;
using mrg::set_error;

namespace mrg {

void group_requests(const std::vector<BatchReq> &in, Grouped *out)
{
    out->reqs.clear();
    out->prefix.clear();
    out->groups.clear();
    out->pos.assign(in.size(), 0);
    out->total_items = 0;
    // wave requests by dtype, in input order, and their output bytes
    std::vector<size_t> wave[3], rows;
    uint64_t bytes[3] = {0, 0, 0};
    for (size_t i = 0; i < in.size(); ++i) {
        const BatchReq &R = in[i];
        if (is_row(R)) {
            rows.push_back(i);
        } else {
            wave[R.dtype].push_back(i);
            bytes[R.dtype] += R.k * R.n * (R.dtype == 2 ? 8 : 4);
        }
    }
    // row items largest first: a row item is whole streams on one wave, one
    // per lane (up to 64 rows of wave_min_bytes), claimed in this order; big
    // ones left for the end would run the launch's tail alone
    auto item_bytes = [&](size_t i) {
        const BatchReq &R = in[i];
        return std::min<uint64_t>(R.k, 64 * (uint64_t)R.spi) * R.n * (R.dtype == 2 ? 8 : 4);
    };
    std::stable_sort(rows.begin(), rows.end(),
                     [&](size_t a, size_t b) { return item_bytes(a) > item_bytes(b); });
    // wave groups with the least output first (shortest-job-first keeps the
    // completion times of most requests low; the run's end does not move)
    std::vector<int> order;
    for (int d = 0; d < 3; ++d)
        if (!wave[d].empty()) order.push_back(d);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return bytes[a] < bytes[b]; });
    if (order.empty() && !rows.empty()) order.push_back(-1);  // rows alone
    for (size_t gi = 0; gi < order.size(); ++gi) {
        const int d = order[gi];
        const bool lead = gi == 0 && !rows.empty();
        Grouped::Group g = {d < 0 ? 0 : d, lead ? kKindRows : kKindWave,
                            (uint32_t)out->reqs.size(), 0, (uint32_t)out->prefix.size(), 0};
        out->prefix.push_back(0);
        auto add = [&](size_t i) {
            out->pos[i] = (uint32_t)out->reqs.size();
            out->reqs.push_back(in[i]);
            g.items += items_of(in[i]);
            out->prefix.push_back(g.items);
            ++g.nreq;
        };
        if (lead)
            for (size_t i : rows) add(i);
        if (d >= 0)
            for (size_t i : wave[d]) add(i);
        out->groups.push_back(g);
        out->total_items += g.items;
    }
}

void plan_batch(const mrg_request *reqs, uint64_t n, const mrg_batch_config &cfg, HostPlan *out)
{
    HostPlan &P = *out;
    P.in.clear();
    P.req_of.clear();
    P.cb_prefix.assign(1, 0);
    P.cb_stream0.clear();
    P.cb_scratch0.clear();
    P.scratch_slots = P.samples = P.bytes = 0;
    for (uint64_t i = 0; i < n; ++i) {
        const mrg_request &q = reqs[i];
        if (!q.count || !q.n_per_stream) continue;
        const uint64_t es = q.dtype == MRG_F64 ? 8 : 4;
        const uint64_t chunk = 64 * (kBatchLaneBytes / es);  // values per wave_fill chunk
        BatchReq R = {};
        R.out = (unsigned char *)q.d_out;
        R.stream0 = q.first;
        R.k = q.count;
        R.n = q.n_per_stream;
        R.sub0 = q.substream0;
        R.dtype = (uint32_t)q.dtype;
        R.flags = (q.flags & MRG_REQ_SUBSTREAMS) ? kReqSubstreams : kReqWriteBack;
        if (R.n * es >= cfg.wave_min_bytes) {
            uint64_t seg = cfg.segment_bytes / es / chunk * chunk;
            if (seg < chunk) seg = chunk;
            R.seg = seg;
            R.segs = (R.n + seg - 1) / seg;
            // streams that fit one segment are packed, about a segment per item
            R.spi = R.segs == 1 ? (uint32_t)std::min<uint64_t>(seg / R.n, 1u << 20) : 1;
            if (!R.spi) R.spi = 1;
            if (R.segs > 1 && (R.flags & kReqWriteBack)) {
                R.scratch0 = P.scratch_slots;
                P.cb_stream0.push_back(R.stream0);
                P.cb_scratch0.push_back(R.scratch0);
                P.cb_prefix.push_back(P.cb_prefix.back() + R.k);
                P.scratch_slots += R.k;
            }
        } else {
            R.seg = 0;
            R.segs = 1;
            R.spi = row_blocks_per_item(R.n, es);
        }
        P.in.push_back(R);
        P.req_of.push_back((uint32_t)i);
        P.samples += R.k * R.n;
        P.bytes += R.k * R.n * es;
    }
    group_requests(P.in, &P.plan);
}

hipError_t launch_grouped(const Grouped &g, const BatchReq *d_reqs, const uint64_t *d_prefix,
                          unsigned long long *d_counters, const BatchArgs &base,
                          uint64_t grid_cap, int engine, hipStream_t st)
{
    for (size_t i = 0; i < g.groups.size(); ++i) {
        const Grouped::Group &G = g.groups[i];
        BatchArgs A = base;
        A.reqs = d_reqs + G.req_off;
        A.prefix = d_prefix + G.prefix_off;
        A.nreq = G.nreq;
        A.total_items = G.items;
        A.counter = d_counters + i;
        if (base.req_done) {
            A.req_done = base.req_done + G.req_off;
        }
        const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min(grid_cap, G.items));
        hipError_t e = launch_batch_group(A, G.dtype, G.kind, grid, engine, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace mrg

struct mrg_batch_s {
    mrg_streamset ss = nullptr;
    int device = -1;
    std::vector<mrg_request> reqs;   // as given (zero-size ones included)
    mrg_batch_config cfg = {};       // effective configuration
    mrg::DeviceTables tabs;
    int engine = 1;

    // plan (host mirror and device copies)
    mrg::Grouped plan;
    std::vector<uint32_t> req_of;    // non-empty request -> input index
    std::vector<uint64_t> cb_prefix, cb_stream0, cb_scratch0;
    uint64_t scratch_slots = 0, samples = 0, bytes = 0;
    mrg::BatchReq *d_reqs = nullptr;
    uint64_t *d_prefix = nullptr;
    uint64_t *d_solo = nullptr;      // [nreq][2]: {0, items of request r}
    uint64_t *d_cb = nullptr;        // cb_prefix | cb_stream0 | cb_scratch0
    unsigned long long *d_counter = nullptr;  // one per group
    unsigned long long *d_stamps = nullptr;   // [nreq] done stamps | start
    uint32_t *d_scratch = nullptr;
    uint64_t grid_cap = 0;

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
                    (void *)b->d_counter, (void *)b->d_stamps, (void *)b->d_scratch})
        if (p) (void)hipFree(p);
    b->d_reqs = nullptr;
    b->d_prefix = b->d_solo = b->d_cb = nullptr;
    b->d_counter = b->d_stamps = nullptr;
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

// Cut the requests into work items under b->cfg, group them and upload the plan.
mrg_status build_plan(mrg_batch b)
{
    free_plan(b);
    mrg::HostPlan hp;
    mrg::plan_batch(b->reqs.data(), b->reqs.size(), b->cfg, &hp);
    b->plan = std::move(hp.plan);
    b->req_of = std::move(hp.req_of);
    b->cb_prefix = std::move(hp.cb_prefix);
    b->cb_stream0 = std::move(hp.cb_stream0);
    b->cb_scratch0 = std::move(hp.cb_scratch0);
    b->scratch_slots = hp.scratch_slots;
    b->samples = hp.samples;
    b->bytes = hp.bytes;
    const std::vector<mrg::BatchReq> &in = hp.in;
    std::vector<uint64_t> solo;
    for (const mrg::BatchReq &R : in) {
        solo.push_back(0);
        solo.push_back(mrg::items_of(R));
    }
    mrg_status st;
    if ((st = upload(&b->d_reqs, b->plan.reqs, "batch requests"))) return st;
    if ((st = upload(&b->d_prefix, b->plan.prefix, "batch prefix"))) return st;
    if ((st = upload(&b->d_solo, solo, "batch solo prefix"))) return st;
    std::vector<uint64_t> cb(b->cb_prefix);
    cb.insert(cb.end(), b->cb_stream0.begin(), b->cb_stream0.end());
    cb.insert(cb.end(), b->cb_scratch0.begin(), b->cb_scratch0.end());
    if ((st = upload(&b->d_cb, cb, "batch copy-back"))) return st;
    hipError_t e = hipMalloc((void **)&b->d_counter, 6 * sizeof(unsigned long long));
    if (e != hipSuccess) return set_error(MRG_ENOMEM, "hipMalloc(counters)");
    e = hipMalloc((void **)&b->d_stamps, (b->plan.reqs.size() + 1) * sizeof(unsigned long long));
    if (e != hipSuccess) return set_error(MRG_ENOMEM, "hipMalloc(completion stamps)");
    if (b->scratch_slots) {
        e = hipMalloc((void **)&b->d_scratch, 6 * b->scratch_slots * sizeof(uint32_t));
        if (e != hipSuccess)
            return set_error(MRG_ENOMEM, "hipMalloc(batch scratch, %llu states)",
                             (unsigned long long)b->scratch_slots);
    }
    b->grid_cap = (uint64_t)b->tabs.cus * b->cfg.waves_per_cu;
    return MRG_OK;
}

mrg::BatchArgs base_args(mrg_batch b)
{
    mrg::BatchArgs A = {};
    A.dynamic = b->cfg.schedule == MRG_SCHEDULE_STATIC ? 0u : 1u;
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
    const uint64_t nr = b->plan.reqs.size();
    A.req_done = b->d_stamps;
    A.t_start = b->d_stamps + nr;
    return A;
}

hipError_t launch_all(mrg_batch b, hipStream_t st)
{
    const mrg::BatchArgs A = base_args(b);
    hipError_t e = mrg::launch_stamp_reset(A.req_done, b->plan.reqs.size(), A.t_start, st);
    if (e != hipSuccess) return e;
    e = mrg::launch_grouped(b->plan, b->d_reqs, b->d_prefix, b->d_counter, A,
                                       b->grid_cap, b->engine, st);
    if (e == hipSuccess) e = mrg::launch_copyback(A, st);
    return e;
}

mrg_status capture(mrg_batch b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    if (!b->plan.total_items) return MRG_OK;
    hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_error(e, "hipStreamBeginCapture");
    hipError_t le = launch_all(b, b->cap_stream);
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
        char what[64];
        snprintf(what, sizeof what, "request %llu: output", (unsigned long long)i);
        if (mrg_status st = mrg::check_device_span(q.d_out, q.count * q.n_per_stream * es,
                                                   ss->device, what))
            return st;
        if (q.flags & MRG_REQ_SUBSTREAMS) {
            if (q.first >= ss->n)
                return set_error(MRG_ERANGE, "request %llu: stream outside the set", (unsigned long long)i);
            if (q.count - 1 > UINT64_MAX - q.substream0)  // substream0 + count - 1 < 2^64
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
    // a substream request reads its stream's state, which a plain request on
    // that stream would overwrite in the same run
    for (uint64_t i = 0; i < n; ++i) {
        const mrg_request &q = reqs[i];
        if (!q.count || !q.n_per_stream || !(q.flags & MRG_REQ_SUBSTREAMS)) continue;
        auto it = std::upper_bound(spans.begin(), spans.end(),
                                   std::make_pair(q.first, UINT64_MAX));
        if (it != spans.begin() && q.first < std::prev(it)->second)
            return set_error(MRG_EINVAL, "request %llu: substreams of stream %llu, which a plain "
                             "request of the batch advances", (unsigned long long)i,
                             (unsigned long long)q.first);
    }
    return MRG_OK;
}

}  // namespace

namespace mrg {

mrg_batch_config batch_config(const mrg_batch_config *c) { return effective(c); }

mrg_status validate_batch(mrg_streamset ss, const mrg_request *reqs, uint64_t n)
{
    return validate(ss, reqs, n);
}

}  // namespace mrg

extern "C" {

mrg_status mrg_batch_create(mrg_batch *out, mrg_streamset ss, const mrg_request *reqs,
                            uint64_t n_reqs, const mrg_batch_config *cfg)
{
    if (!out) return set_error(MRG_EINVAL, "null output handle");
    *out = nullptr;
    mrg_status st = mrg::check_streamset(ss);
    if (st) return st;
    if (ss->gen != 0) return set_error(MRG_EINVAL, "batches take MRG32k3a stream sets only");
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
    if (!b->plan.total_items) return MRG_OK;
    hipError_t e = launch_all(b, (hipStream_t)stream);
    return e == hipSuccess ? MRG_OK : hip_error(e, "batch kernel launch");
}

mrg_status mrg_batch_run_per_request(mrg_batch b, void *stream)
{
    if (!b) return set_error(MRG_EINVAL, "null batch");
    for (size_t r = 0; r < b->req_of.size(); ++r) {
        const mrg_request &q = b->reqs[b->req_of[r]];
        mrg_status st;
        if (q.flags & MRG_REQ_SUBSTREAMS) {
            // the batch kernel restricted to this one request
            const uint32_t p = b->plan.pos[r];
            const mrg::BatchReq &R = b->plan.reqs[p];
            mrg::BatchArgs A = base_args(b);
            A.reqs = b->d_reqs + p;
            A.prefix = b->d_solo + 2 * r;
            A.nreq = 1;
            A.total_items = mrg::items_of(R);
            A.counter = b->d_counter;
            A.req_done = A.t_start = nullptr;  // stamps belong to batch runs
            const unsigned grid =
                (unsigned)std::max<uint64_t>(1, std::min(b->grid_cap, A.total_items));
            hipError_t e = mrg::launch_batch_group(
                A, (int)R.dtype, mrg::is_row(R) ? mrg::kKindRows : mrg::kKindWave, grid, b->engine,
                (hipStream_t)stream);
            st = e == hipSuccess ? MRG_OK : hip_error(e, "batch kernel launch");
        } else {
            st = mrg_fill(b->ss, q.first, q.count, q.n_per_stream, (mrg_dtype)q.dtype,
                          MRG_STREAM_MAJOR, q.d_out, stream);
        }
        if (st) return st;
    }
    return MRG_OK;
}

mrg_status mrg_batch_request_times(mrg_batch b, void *stream, double *h_ms)
{
    if (!b || !h_ms) return set_error(MRG_EINVAL, "null argument");
    const size_t nr = b->plan.reqs.size();
    std::vector<unsigned long long> st(nr + 1);
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e == hipSuccess)
        e = hipMemcpy(st.data(), b->d_stamps, st.size() * sizeof(unsigned long long),
                      hipMemcpyDeviceToHost);
    int khz = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, b->device);
    if (e != hipSuccess) return hip_error(e, "reading completion stamps");
    if (khz <= 0) return set_error(MRG_EHIP, "no wall clock rate");
    for (size_t i = 0; i < b->reqs.size(); ++i) h_ms[i] = 0.0;
    const unsigned long long t0 = st[nr];
    for (size_t r = 0; r < b->req_of.size(); ++r) {
        const unsigned long long t = st[b->plan.pos[r]];
        h_ms[b->req_of[r]] = t >= t0 ? (double)(t - t0) / (double)khz : 0.0;
    }
    return MRG_OK;
}

mrg_status mrg_batch_info(mrg_batch b, mrg_batch_info_t *info)
{
    if (!b || !info) return set_error(MRG_EINVAL, "null argument");
    info->requests = b->req_of.size();
    info->items = b->plan.total_items;
    info->samples = b->samples;
    info->bytes = b->bytes;
    info->grid = (uint32_t)std::max<uint64_t>(1, std::min(b->grid_cap, b->plan.total_items));
    info->scratch_states = b->scratch_slots;
    info->config = b->cfg;
    return MRG_OK;
}

mrg_status mrg_batch_plan_groups(const mrg_request *reqs, uint64_t n_reqs,
                                 const mrg_batch_config *cfg, mrg_plan_group *groups,
                                 uint32_t *n_groups, uint64_t *pos, uint64_t *items)
{
    if ((!reqs && n_reqs) || !groups || !n_groups) return set_error(MRG_EINVAL, "null argument");
    for (uint64_t i = 0; i < n_reqs; ++i) {
        const mrg_request &q = reqs[i];
        if (q.dtype != MRG_U32 && q.dtype != MRG_F32 && q.dtype != MRG_F64)
            return set_error(MRG_EINVAL, "request %llu: unknown dtype %d", (unsigned long long)i,
                             (int)q.dtype);
        if (q.flags & ~(uint32_t)MRG_REQ_SUBSTREAMS)
            return set_error(MRG_EINVAL, "request %llu: unknown flags", (unsigned long long)i);
    }
    mrg::HostPlan P;
    mrg::plan_batch(reqs, n_reqs, mrg::batch_config(cfg), &P);
    const mrg::Grouped &g = P.plan;
    *n_groups = (uint32_t)g.groups.size();
    for (size_t k = 0; k < g.groups.size(); ++k) {
        const mrg::Grouped::Group &G = g.groups[k];
        mrg_plan_group &o = groups[k];
        o.dtype = G.dtype;
        o.rows = G.kind == mrg::kKindRows ? 1 : 0;
        o.requests = G.nreq;
        o.items = G.items;
        o.row_items = 0;
        o.bytes = 0;
        for (uint32_t r = G.req_off; r < G.req_off + G.nreq; ++r) {
            const mrg::BatchReq &R = g.reqs[r];
            if (mrg::is_row(R)) o.row_items += mrg::items_of(R);
            o.bytes += R.k * R.n * (R.dtype == 2 ? 8 : 4);
        }
    }
    if (pos)
        for (uint64_t i = 0; i < n_reqs; ++i) pos[i] = UINT64_MAX;
    if (items)
        for (uint64_t i = 0; i < n_reqs; ++i) items[i] = 0;
    for (size_t r = 0; r < P.req_of.size(); ++r) {
        const uint64_t i = P.req_of[r];
        if (pos) pos[i] = g.pos[r];
        if (items) items[i] = mrg::items_of(P.in[r]);
    }
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
        (void)hipStreamSynchronize(st);
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
