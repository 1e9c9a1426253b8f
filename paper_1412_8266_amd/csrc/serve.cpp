// Serving engine: continuous batching of generation requests from many
// clients.
//
// Every client owns one stream of a resident stream set (its state never
// changes) and a substream cursor kept on the host.  A request of client c
// for k streams of n values gets the client's next k substreams (sec. 4.1:
// substreams of 2^76 values), so requests of one client never depend on each
// other and can run concurrently.  A scheduler thread admits queued requests
// in arrival order within two size classes (large requests queue apart and
// run on their own quarter of the HIP streams) while the output arena has room
// (first fit), launches each
// admitted group ("tick": one persistent batch kernel per launch group, batch.h)
// on the next of several HIP streams -- ticks overlap on the device -- and
// retires ticks by polling their completion events.  Latency is measured from submission to the
// moment the scheduler observes the tick's event complete.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "batch.h"
#include "internal.h"

using mrg::hip_error;
using mrg::set_error;

namespace {

using Clock = std::chrono::steady_clock;

double now_s()
{
    return std::chrono::duration<double>(Clock::now().time_since_epoch()).count();
}

struct Req {
    uint64_t ticket;
    uint64_t client, k, n;
    int dtype;
    uint64_t bytes;
    double t_submit;
    double t_admit = 0, t_done = 0;
    uint64_t offset = 0;   // arena offset
    uint64_t sub0 = 0;     // first substream
};

// First-fit allocator over [0, size) with coalescing frees.
class Arena {
public:
    explicit Arena(uint64_t size) : size_(size) { free_[0] = size; }
    bool alloc(uint64_t bytes, uint64_t *off)
    {
        bytes = (bytes + 255) / 256 * 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const uint64_t rest = it->second - bytes, at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes)
    {
        bytes = (bytes + 255) / 256 * 256;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint64_t used() const { return used_; }
    uint64_t size() const { return size_; }

private:
    uint64_t size_, used_ = 0;
    std::map<uint64_t, uint64_t> free_;
};

struct Slot {  // one tick in flight
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    mrg::BatchReq *d_reqs = nullptr;
    uint64_t *d_prefix = nullptr;
    unsigned long long *d_counter = nullptr;  // one per launch group (at most 3)
    mrg::BatchReq *h_reqs = nullptr;  // pinned staging
    uint64_t *h_prefix = nullptr;
    std::vector<Req> reqs;
    mrg::Grouped plan;
    bool busy = false;
};

}  // namespace

struct mrg_server_s {
    mrg_server_config cfg = {};
    int device = -1;
    mrg_streamset clients = nullptr;
    mrg::DeviceTables tabs;
    int engine = 1;
    unsigned char *d_arena = nullptr;
    Arena *arena = nullptr;
    std::vector<uint64_t> cursor;  // next substream of each client
    std::vector<Slot> slots;
    size_t next_slot[2] = {0, 0};  // round robin within each slot pool
    size_t n_small_slots = 0;      // slots [0, n) serve small requests, the rest large ones

    std::mutex mu;
    std::condition_variable cv;
    std::deque<Req> pending[2];    // queued small (0) and large (1) requests
    std::deque<Req> done;             // finished, not yet taken by poll
    std::map<uint64_t, Req> held;     // finished, output held until release
    uint64_t next_ticket = 1;
    uint64_t inflight_reqs = 0;
    std::atomic<bool> stop{false};
    std::thread worker;
    mrg_status worker_status = MRG_OK;
    std::string worker_error;
    uint64_t ticks = 0, completed = 0, samples_done = 0, bytes_done = 0;
};

namespace {

mrg::BatchReq to_batch_req(mrg_server s, const Req &r)
{
    mrg::BatchReq R = {};
    const uint64_t es = r.dtype == MRG_F64 ? 8 : 4;
    R.out = s->d_arena + r.offset;
    R.stream0 = r.client;
    R.k = r.k;
    R.n = r.n;
    R.sub0 = r.sub0;
    R.dtype = (uint32_t)r.dtype;
    R.flags = mrg::kReqSubstreams;
    if (r.n * es >= 16 * 1024) {
        const uint64_t chunk = 64 * (mrg::kBatchLaneBytes / es);
        uint64_t seg = (256 * 1024) / es / chunk * chunk;
        R.seg = seg;
        R.segs = (r.n + seg - 1) / seg;
        R.spi = R.segs == 1 ? (uint32_t)std::max<uint64_t>(1, seg / r.n) : 1;
    } else {
        R.seg = 0;
        R.segs = 1;
        R.spi = mrg::row_blocks_per_item(r.n, es);
    }
    return R;
}

// Launch the admitted requests of `slot` (scheduler thread): one persistent
// kernel per launch group, all on the slot's stream.
mrg_status launch_tick(mrg_server s, Slot &slot)
{
    std::vector<mrg::BatchReq> in(slot.reqs.size());
    for (size_t i = 0; i < slot.reqs.size(); ++i) in[i] = to_batch_req(s, slot.reqs[i]);
    mrg::group_requests(in, &slot.plan);
    const size_t nr = slot.plan.reqs.size(), np = slot.plan.prefix.size();
    std::memcpy(slot.h_reqs, slot.plan.reqs.data(), nr * sizeof(mrg::BatchReq));
    std::memcpy(slot.h_prefix, slot.plan.prefix.data(), np * sizeof(uint64_t));
    hipError_t e = hipMemcpyAsync(slot.d_reqs, slot.h_reqs, nr * sizeof(mrg::BatchReq),
                                  hipMemcpyHostToDevice, slot.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(slot.d_prefix, slot.h_prefix, np * sizeof(uint64_t),
                           hipMemcpyHostToDevice, slot.stream);
    if (e != hipSuccess) return hip_error(e, "tick upload");
    mrg::BatchArgs A = {};
    A.dynamic = 1;
    A.planes = s->clients->d_planes;
    A.plane_stride = s->clients->n;
    A.table = s->tabs.table;
    A.lane_tab = s->tabs.lane_tab;
    const uint64_t cap = (uint64_t)s->tabs.cus * s->cfg.waves_per_cu;
    e = mrg::launch_grouped(slot.plan, slot.d_reqs, slot.d_prefix, slot.d_counter, A, cap,
                            s->engine, slot.stream);
    if (e == hipSuccess) e = hipEventRecord(slot.done, slot.stream);
    if (e != hipSuccess) return hip_error(e, "tick launch");
    slot.busy = true;
    return MRG_OK;
}

// A tick that failed to launch or to complete: its requests are dropped (their
// arena space returned, no longer in flight) and the slot freed.  Called with
// the server lock held.
void drop_tick(mrg_server s, Slot &slot)
{
    for (const Req &r : slot.reqs) s->arena->release(r.offset, r.bytes);
    s->inflight_reqs -= slot.reqs.size();
    slot.reqs.clear();
    slot.busy = false;
}

void scheduler(mrg_server s)
{
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // retire finished ticks
        bool progressed = false;
        for (Slot &slot : s->slots) {
            if (!slot.busy) continue;
            hipError_t q = hipEventQuery(slot.done);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) {
                s->worker_status = MRG_EHIP;
                s->worker_error = hipGetErrorString(q);
                s->stop = true;
                drop_tick(s, slot);  // its outputs are lost; let the scheduler exit
                continue;
            }
            const double t = now_s();
            for (Req &r : slot.reqs) {
                r.t_done = t;
                ++s->completed;
                s->samples_done += r.k * r.n;
                s->bytes_done += r.bytes;
                if (s->cfg.auto_release) s->arena->release(r.offset, r.bytes);
                else s->held[r.ticket] = r;
                s->done.push_back(r);
            }
            s->inflight_reqs -= slot.reqs.size();
            slot.reqs.clear();
            slot.busy = false;
            progressed = true;
        }
        if (s->stop && s->inflight_reqs == 0) break;
        // admit each size class into the next free slot of its own pool, so
        // that small requests never wait in a tick behind a large one
        for (int cls = 0; cls < 2 && !s->stop; ++cls) {
            const size_t lo = cls ? s->n_small_slots : 0;
            const size_t pool = cls ? s->slots.size() - s->n_small_slots : s->n_small_slots;
            Slot *free_slot = nullptr;
            for (size_t i = 0; i < pool; ++i) {
                const size_t at = (s->next_slot[cls] + i) % pool;
                Slot &c = s->slots[lo + at];
                if (!c.busy) {
                    free_slot = &c;
                    s->next_slot[cls] = (at + 1) % pool;
                    break;
                }
            }
            if (free_slot) {
                std::deque<Req> &q = s->pending[cls];
                while (!q.empty() && free_slot->reqs.size() < s->cfg.max_batch) {
                    Req &r = q.front();
                    uint64_t off;
                    if (!s->arena->alloc(r.bytes, &off)) break;  // head waits for memory
                    r.offset = off;
                    r.sub0 = s->cursor[r.client];
                    s->cursor[r.client] += r.k;
                    r.t_admit = now_s();
                    free_slot->reqs.push_back(r);
                    q.pop_front();
                }
                if (!free_slot->reqs.empty()) {
                    s->inflight_reqs += free_slot->reqs.size();
                    ++s->ticks;
                    // the slot belongs to this thread alone: launch without the
                    // lock, so that submissions are not held up by the launches
                    lk.unlock();
                    const mrg_status st = launch_tick(s, *free_slot);
                    const std::string err = st ? mrg_last_error() : "";
                    lk.lock();
                    if (st) {
                        s->worker_status = st;
                        s->worker_error = err;
                        s->stop = true;
                        drop_tick(s, *free_slot);
                    }
                    progressed = true;
                }
            }
        }
        if (!progressed) {
            // nothing to do: wait briefly for arrivals or device progress
            s->cv.wait_for(lk, std::chrono::microseconds(s->inflight_reqs ? 20 : 200));
        }
    }
}

}  // namespace

extern "C" {

mrg_status mrg_server_create(mrg_server *out, const mrg_server_config *cfg_in)
{
    if (!out || !cfg_in) return set_error(MRG_EINVAL, "null argument");
    *out = nullptr;
    mrg_server_config cfg = *cfg_in;
    if (!cfg.n_clients) return set_error(MRG_ERANGE, "n_clients must be >= 1");
    // the arena hands out 256-byte-aligned blocks of whole 256-byte units, so
    // only whole units of it can ever be used
    cfg.arena_bytes = cfg.arena_bytes / 256 * 256;
    if (!cfg.arena_bytes) return set_error(MRG_ERANGE, "arena_bytes must be at least 256");
    if (!cfg.max_inflight) cfg.max_inflight = 8;
    if (!cfg.max_batch) cfg.max_batch = 4096;
    if (!cfg.waves_per_cu) cfg.waves_per_cu = 8;
    if (!cfg.big_request_bytes) cfg.big_request_bytes = 64ull << 20;
    if (cfg.max_inflight > 64) return set_error(MRG_ERANGE, "max_inflight above 64");
    if (cfg.max_batch > (1u << 20)) return set_error(MRG_ERANGE, "max_batch above 2^20");
    auto *s = new (std::nothrow) mrg_server_s;
    if (!s) return set_error(MRG_ENOMEM, "host allocation");
    s->cfg = cfg;
    mrg_status st = mrg_streamset_create_seed64(&s->clients, cfg.n_clients, cfg.first_stream,
                                                cfg.master_seed, nullptr);
    if (st) {
        delete s;
        return st;
    }
    s->device = s->clients->device;
    s->engine = mrg::current_tuning().engine;
    if ((st = mrg::device_tables(s->device, &s->tabs))) {
        mrg_streamset_destroy(s->clients);
        delete s;
        return st;
    }
    hipError_t e = hipMalloc(&s->d_arena, cfg.arena_bytes);
    if (e != hipSuccess) {
        mrg_streamset_destroy(s->clients);
        delete s;
        return set_error(MRG_ENOMEM, "hipMalloc(arena of %llu bytes)",
                         (unsigned long long)cfg.arena_bytes);
    }
    s->arena = new Arena(cfg.arena_bytes);
    s->cursor.assign(cfg.n_clients, 0);
    s->slots.resize(cfg.max_inflight);
    // a quarter of the slots (at least one) for large requests, unless one class
    s->n_small_slots = cfg.big_request_bytes == UINT64_MAX || cfg.max_inflight < 2
                           ? cfg.max_inflight
                           : cfg.max_inflight - std::max<uint32_t>(1, cfg.max_inflight / 4);
    for (Slot &slot : s->slots) {
        e = hipStreamCreateWithFlags(&slot.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&slot.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipMalloc(&slot.d_reqs, cfg.max_batch * sizeof(mrg::BatchReq));
        if (e == hipSuccess) e = hipMalloc(&slot.d_prefix, (cfg.max_batch + 6) * sizeof(uint64_t));
        if (e == hipSuccess) e = hipMalloc(&slot.d_counter, 6 * sizeof(unsigned long long));
        if (e == hipSuccess)
            e = hipHostMalloc(&slot.h_reqs, cfg.max_batch * sizeof(mrg::BatchReq), 0);
        if (e == hipSuccess)
            e = hipHostMalloc(&slot.h_prefix, (cfg.max_batch + 6) * sizeof(uint64_t), 0);
        if (e != hipSuccess) {
            st = hip_error(e, "server slot setup");
            break;
        }
    }
    e = hipDeviceSynchronize();  // client states are ready before any tick
    if (!st && e != hipSuccess) st = hip_error(e, "hipDeviceSynchronize");
    if (st) {
        mrg_server_destroy(s);
        return st;
    }
    s->worker = std::thread(scheduler, s);
    *out = s;
    return MRG_OK;
}

mrg_status mrg_server_submit(mrg_server s, uint64_t client, uint64_t n_streams,
                             uint64_t n_per_stream, int32_t dtype, uint64_t *ticket)
{
    if (!s) return set_error(MRG_EINVAL, "null server");
    if (client >= s->cfg.n_clients) return set_error(MRG_ERANGE, "client out of range");
    if (dtype != MRG_U32 && dtype != MRG_F32 && dtype != MRG_F64)
        return set_error(MRG_EINVAL, "unknown dtype");
    if (!n_streams || !n_per_stream) return set_error(MRG_EINVAL, "empty request");
    const uint64_t es = dtype == MRG_F64 ? 8 : 4;
    // compared as the arena will hold it (rounded up to 256 bytes), so that a
    // request admitted here always fits once the arena is empty
    if (n_per_stream > s->cfg.arena_bytes / es / n_streams ||
        (n_streams * n_per_stream * es + 255) / 256 * 256 > s->cfg.arena_bytes)
        return set_error(MRG_ERANGE, "request larger than the arena");
    Req r;
    r.client = client;
    r.k = n_streams;
    r.n = n_per_stream;
    r.dtype = dtype;
    r.bytes = n_streams * n_per_stream * es;
    r.t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return set_error(MRG_EHIP, "server stopped: %s", s->worker_error.c_str());
        r.ticket = s->next_ticket++;
        s->pending[r.bytes >= s->cfg.big_request_bytes && s->n_small_slots < s->slots.size()]
            .push_back(r);
    }
    s->cv.notify_one();
    if (ticket) *ticket = r.ticket;
    return MRG_OK;
}

mrg_status mrg_server_poll(mrg_server s, mrg_server_result *out, uint64_t max_out,
                           uint64_t *n_out)
{
    if (!s || !n_out || (max_out && !out)) return set_error(MRG_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    uint64_t n = std::min<uint64_t>(max_out, s->done.size());
    for (uint64_t i = 0; i < n; ++i) {
        const Req &r = s->done[i];
        mrg_server_result &o = out[i];
        o.ticket = r.ticket;
        o.client = r.client;
        o.n_streams = r.k;
        o.n_per_stream = r.n;
        o.substream0 = r.sub0;
        o.dtype = r.dtype;
        o.d_out = s->cfg.auto_release ? nullptr : (void *)(s->d_arena + r.offset);
        o.latency_s = r.t_done - r.t_submit;
        o.queue_s = r.t_admit - r.t_submit;
        o.t_submit = r.t_submit;
    }
    s->done.erase(s->done.begin(), s->done.begin() + n);
    *n_out = n;
    return s->worker_status;
}

mrg_status mrg_server_release(mrg_server s, uint64_t ticket)
{
    if (!s) return set_error(MRG_EINVAL, "null server");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->held.find(ticket);
        if (it == s->held.end()) return set_error(MRG_EINVAL, "ticket not held");
        s->arena->release(it->second.offset, it->second.bytes);
        s->held.erase(it);
    }
    s->cv.notify_one();
    return MRG_OK;
}

mrg_status mrg_server_copy_output(mrg_server s, uint64_t ticket, void *h_dst, uint64_t bytes)
{
    if (!s || (bytes && !h_dst)) return set_error(MRG_EINVAL, "null argument");
    uint64_t off, size;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->held.find(ticket);
        if (it == s->held.end()) return set_error(MRG_EINVAL, "ticket not held");
        off = it->second.offset;
        size = it->second.bytes;
    }
    if (bytes > size) return set_error(MRG_ERANGE, "copy larger than the output");
    hipError_t e = hipMemcpy(h_dst, s->d_arena + off, bytes, hipMemcpyDeviceToHost);
    return e == hipSuccess ? MRG_OK : hip_error(e, "hipMemcpy(output)");
}

mrg_status mrg_server_stats(mrg_server s, mrg_server_stats_t *st)
{
    if (!s || !st) return set_error(MRG_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    st->pending = s->pending[0].size() + s->pending[1].size();
    st->inflight = s->inflight_reqs;
    st->completed = s->completed;
    st->ticks = s->ticks;
    st->samples = s->samples_done;
    st->bytes = s->bytes_done;
    st->arena_used = s->arena->used();
    st->arena_bytes = s->arena->size();
    return s->worker_status;
}

mrg_status mrg_server_drain(mrg_server s, double timeout_s)
{
    if (!s) return set_error(MRG_EINVAL, "null server");
    const double t_end = now_s() + timeout_s;
    for (;;) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            if (s->worker_status) return s->worker_status;
            if (s->pending[0].empty() && s->pending[1].empty() && s->inflight_reqs == 0)
                return MRG_OK;
            // nothing in flight but the head still queued: its memory is held
            // by outputs that only mrg_server_release can free
            if (s->inflight_reqs == 0 && !s->held.empty() && now_s() > t_end - timeout_s + 0.05)
                return set_error(MRG_EBUSY, "queued requests wait for held outputs");
        }
        if (now_s() > t_end) return set_error(MRG_EBUSY, "drain timed out");
        std::this_thread::sleep_for(std::chrono::microseconds(100));
    }
}

mrg_status mrg_server_run_trace(mrg_server s, const mrg_arrival *arr, uint64_t n,
                                double time_scale, double *wall_s)
{
    if (!s || (n && !arr)) return set_error(MRG_EINVAL, "null argument");
    if (!(time_scale > 0)) time_scale = 1.0;
    const double t0 = now_s();
    for (uint64_t i = 0; i < n; ++i) {
        const double due = t0 + arr[i].t * time_scale;
        double t;
        while ((t = now_s()) < due) {
            if (due - t > 200e-6) std::this_thread::sleep_for(std::chrono::microseconds(50));
        }
        mrg_status st = mrg_server_submit(s, arr[i].client, arr[i].n_streams, arr[i].n_per_stream,
                                          arr[i].dtype, nullptr);
        if (st) return st;
    }
    mrg_status st = mrg_server_drain(s, 3600.0);
    if (wall_s) *wall_s = now_s() - t0;
    return st;
}

mrg_status mrg_server_client_state(mrg_server s, uint64_t client, uint32_t out6[6],
                                   uint64_t *next_substream)
{
    if (!s || !out6) return set_error(MRG_EINVAL, "null argument");
    if (client >= s->cfg.n_clients) return set_error(MRG_ERANGE, "client out of range");
    mrg_status st = mrg_get_states(s->clients, client, 1, out6, nullptr);
    if (st) return st;
    if (next_substream) {
        std::lock_guard<std::mutex> lk(s->mu);
        *next_substream = s->cursor[client];
    }
    return MRG_OK;
}

mrg_status mrg_server_destroy(mrg_server s)
{
    if (!s) return MRG_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->pending[0].clear();
        s->pending[1].clear();
    }
    s->cv.notify_one();
    if (s->worker.joinable()) s->worker.join();
    (void)hipDeviceSynchronize();
    for (Slot &slot : s->slots) {
        if (slot.stream) (void)hipStreamDestroy(slot.stream);
        if (slot.done) (void)hipEventDestroy(slot.done);
        if (slot.d_reqs) (void)hipFree(slot.d_reqs);
        if (slot.d_prefix) (void)hipFree(slot.d_prefix);
        if (slot.d_counter) (void)hipFree(slot.d_counter);
        if (slot.h_reqs) (void)hipHostFree(slot.h_reqs);
        if (slot.h_prefix) (void)hipHostFree(slot.h_prefix);
    }
    if (s->d_arena) (void)hipFree(s->d_arena);
    delete s->arena;
    if (s->clients) mrg_streamset_destroy(s->clients);
    delete s;
    return MRG_OK;
}

}  // extern "C"
