// C ABI of the MRG32k3a stream library: argument validation, host-side jump
// matrices and tables, device memory of stream sets, kernel launches.
//
// Host initialisation before any kernel (sec. 5.1): creating a stream set
// allocates its device state and computes every stream's starting state on
// the device; release frees it.  Streams and substreams follow sec. 4.1 and
// the jump ahead of sec. 2.3 (matrix powers mod m).
#include <hip/hip_runtime.h>

#include <array>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "mrg_arith.hpp"

namespace {
thread_local std::string g_last_error;
}

namespace mrg {

mrg_status set_error(mrg_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

mrg_status hip_error(hipError_t e, const char *what)
{
    return set_error(MRG_EHIP, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace mrg

namespace {

using mrg::set_error;
using mrg::hip_error;

// ---- host jump matrices (sec. 2.3) ---------------------------------------
using Mat = std::array<uint32_t, 9>;

Mat identity() { return {1, 0, 0, 0, 1, 0, 0, 0, 1}; }

uint64_t modulus(int c) { return c == 0 ? mrg::M1 : mrg::M2; }

// Companion matrix of component c on the column (x[n-3], x[n-2], x[n-1]).
Mat companion(int c)
{
    Mat A = {0, 1, 0, 0, 0, 1, 0, 0, 0};
    if (c == 0) {
        A[6] = mrg::M1 - mrg::A13N;
        A[7] = mrg::A12;
    } else {
        A[6] = mrg::M2 - mrg::A23N;
        A[8] = mrg::A21;
    }
    return A;
}

Mat mul(const Mat &X, const Mat &Y, uint64_t m)
{
    Mat R;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            unsigned __int128 acc = 0;
            for (int k = 0; k < 3; ++k) acc += (unsigned __int128)X[3 * i + k] * Y[3 * k + j];
            R[3 * i + j] = (uint32_t)(acc % m);
        }
    return R;
}

Mat power(int c, const uint64_t e[3])
{
    const uint64_t m = modulus(c);
    Mat R = identity(), B = companion(c);
    int top = 191;
    while (top >= 0 && !((e[top / 64] >> (top % 64)) & 1u)) --top;
    for (int b = 0; b <= top; ++b) {
        if ((e[b / 64] >> (b % 64)) & 1u) R = mul(R, B, m);
        if (b < top) B = mul(B, B, m);
    }
    return R;
}

// T[c][w][d] = A_c^(d * 16^w), d = 0 the identity.
std::vector<uint32_t> build_tables()
{
    std::vector<uint32_t> t(mrg::kTableWords);
    for (int c = 0; c < 2; ++c) {
        const uint64_t m = modulus(c);
        Mat base = companion(c);  // A^(16^w)
        for (int w = 0; w < mrg::kTableWindows; ++w) {
            Mat cur = identity();
            for (int d = 0; d < 16; ++d) {
                std::memcpy(&t[((c * mrg::kTableWindows + w) * 16 + d) * 9], cur.data(), 36);
                cur = mul(cur, base, m);
            }
            // cur = base^16 = A^(16^(w+1))
            base = cur;
        }
    }
    return t;
}

const std::vector<uint32_t> &host_tables()
{
    static const std::vector<uint32_t> t = build_tables();
    return t;
}

// ---- per-device context ----------------------------------------------------
struct DevCtx {
    uint32_t *d_table = nullptr;     // windowed jump tables
    uint32_t *d_lane_tab = nullptr;  // [kNumLaneSegs][64][18]: A^(l*L) for L in kLaneSegs
    int cus = 256;                   // compute units of the device
};

// A^(l*L) for l in [0, 64) and each lane-segment length L, both components.
std::vector<uint32_t> build_lane_tables()
{
    std::vector<uint32_t> t(mrg::kNumLaneTabs * 64 * 18);
    for (int k = 0; k < mrg::kNumLaneTabs; ++k) {
        const uint64_t L = k == mrg::kHeadTable ? 1 : (uint64_t)(16 * (k + 1));
        for (int l = 0; l < 64; ++l) {
            const uint64_t e[3] = {L * (uint64_t)l, 0, 0};
            for (int c = 0; c < 2; ++c) {
                const Mat P = power(c, e);
                std::memcpy(&t[(k * 64 + l) * 18 + 9 * c], P.data(), 36);
            }
        }
    }
    return t;
}

std::mutex g_mu;
std::map<int, DevCtx> g_dev;
mrg::FillTuning g_tune;  // process-wide kernel tuning (guarded by g_mu)

mrg::FillTuning tuning()
{
    std::lock_guard<std::mutex> lk(g_mu);
    return g_tune;
}

mrg_status current_device(int *dev)
{
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0) return set_error(MRG_ENODEV, "no HIP device available");
    e = hipGetDevice(dev);
    if (e != hipSuccess) return hip_error(e, "hipGetDevice");
    return MRG_OK;
}

mrg_status device_ctx(int dev, DevCtx **out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_dev.find(dev);
    if (it != g_dev.end()) {
        *out = &it->second;
        return MRG_OK;
    }
    const std::vector<uint32_t> &t = host_tables();
    DevCtx ctx;
    hipError_t e = hipMalloc(&ctx.d_table, t.size() * sizeof(uint32_t));
    if (e != hipSuccess) return set_error(MRG_ENOMEM, "hipMalloc(jump tables): %s", hipGetErrorString(e));
    e = hipMemcpy(ctx.d_table, t.data(), t.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(ctx.d_table);
        return hip_error(e, "hipMemcpy(jump tables)");
    }
    const std::vector<uint32_t> lt = build_lane_tables();
    e = hipMalloc(&ctx.d_lane_tab, lt.size() * sizeof(uint32_t));
    if (e != hipSuccess) {
        (void)hipFree(ctx.d_table);
        return set_error(MRG_ENOMEM, "hipMalloc(lane tables): %s", hipGetErrorString(e));
    }
    e = hipMemcpy(ctx.d_lane_tab, lt.data(), lt.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(ctx.d_table);
        (void)hipFree(ctx.d_lane_tab);
        return hip_error(e, "hipMemcpy(lane tables)");
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
        ctx.cus = cus;
    auto res = g_dev.emplace(dev, ctx);
    *out = &res.first->second;
    return MRG_OK;
}

bool state_ok(const uint32_t *s)
{
    if (s[0] >= mrg::M1 || s[1] >= mrg::M1 || s[2] >= mrg::M1) return false;
    if (s[3] >= mrg::M2 || s[4] >= mrg::M2 || s[5] >= mrg::M2) return false;
    if ((s[0] | s[1] | s[2]) == 0u || (s[3] | s[4] | s[5]) == 0u) return false;
    return true;
}

}  // namespace

namespace mrg {

FillTuning current_tuning() { return tuning(); }

mrg_status current_device_id(int *dev) { return current_device(dev); }

mrg_status device_tables(int dev, DeviceTables *out)
{
    DevCtx *ctx;
    mrg_status st = device_ctx(dev, &ctx);
    if (st) return st;
    out->table = ctx->d_table;
    out->lane_tab = ctx->d_lane_tab;
    out->cus = ctx->cus;
    return MRG_OK;
}

mrg_status check_streamset(mrg_streamset ss)
{
    if (!ss || !ss->d_planes) return set_error(MRG_EINVAL, "null stream set");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != ss->device)
        return set_error(MRG_EINVAL, "stream set lives on device %d, current device is %d", ss->device, dev);
    return MRG_OK;
}

mrg_status check_device_span(const void *p, uint64_t bytes, int dev, const char *what)
{
    hipPointerAttribute_t a;
    hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();  // keep the failed lookup from reaching a later launch check
        return set_error(MRG_EINVAL, "%s (%p) is not memory known to HIP: %s", what, p,
                         hipGetErrorString(e));
    }
    const bool managed = a.type == hipMemoryTypeManaged || a.isManaged;
    if (!managed && !(a.type == hipMemoryTypeDevice && a.device == dev))
        return set_error(MRG_EINVAL, "%s (%p) is not device memory of device %d (memory type %d, "
                         "device %d)", what, p, dev, (int)a.type, a.device);
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    e = hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return MRG_OK;  // no extent known: the type check above is all there is
    }
    const uint64_t off = (uint64_t)((uintptr_t)p - (uintptr_t)base);
    if (off > size || bytes > size - off)
        return set_error(MRG_ERANGE, "%s (%p, %llu bytes) extends past the end of its allocation "
                         "(%llu bytes at %p)", what, p, (unsigned long long)bytes,
                         (unsigned long long)size, (void *)base);
    return MRG_OK;
}

mrg_status check_range(mrg_streamset ss, uint64_t first, uint64_t count)
{
    if (first > ss->n || count > ss->n - first)
        return set_error(MRG_ERANGE, "streams [%llu, %llu+%llu) outside the set of %llu",
                    (unsigned long long)first, (unsigned long long)first,
                    (unsigned long long)count, (unsigned long long)ss->n);
    // one lane per stream, gridDim.x < 2^31 blocks of 64
    if (count > ((uint64_t)1 << 36))
        return set_error(MRG_ERANGE, "count %llu above the per-call limit 2^36", (unsigned long long)count);
    return MRG_OK;
}

}  // namespace mrg

namespace {

using mrg::check_range;
mrg_status check_set(mrg_streamset ss) { return mrg::check_streamset(ss); }

int bit_length(uint64_t v)
{
    int b = 0;
    while (v) { ++b; v >>= 1; }
    return b;
}

// Validated size, device context and state planes of a new stream set.
mrg_status new_streamset(uint64_t n_streams, uint64_t first_stream, mrg_streamset *out,
                         DevCtx **ctx_out)
{
    if (n_streams == 0) return set_error(MRG_ERANGE, "n_streams must be >= 1");
    if (n_streams - 1 > UINT64_MAX - first_stream)
        return set_error(MRG_ERANGE, "first_stream + n_streams exceeds 2^64");
    if (n_streams > ((uint64_t)1 << 36))
        return set_error(MRG_ERANGE, "n_streams above the limit 2^36");
    int dev;
    mrg_status st = current_device(&dev);
    if (st) return st;
    if ((st = device_ctx(dev, ctx_out))) return st;
    auto *ss = new (std::nothrow) mrg_streamset_s;
    if (!ss) return set_error(MRG_ENOMEM, "host allocation");
    ss->device = dev;
    ss->n = n_streams;
    ss->first = first_stream;
    hipError_t e = hipMalloc(&ss->d_planes, 6 * n_streams * sizeof(uint32_t));
    if (e != hipSuccess) {
        delete ss;
        return set_error(MRG_ENOMEM, "hipMalloc(%llu states): %s", (unsigned long long)n_streams,
                         hipGetErrorString(e));
    }
    *out = ss;
    return MRG_OK;
}

// A^e for both components as kernel arguments.
mrg::JumpMatrices jump_matrices(const uint64_t e[3])
{
    mrg::JumpMatrices J;
    const Mat P1 = power(0, e), P2 = power(1, e);
    std::memcpy(J.m, P1.data(), 36);
    std::memcpy(J.m + 9, P2.data(), 36);
    return J;
}

}  // namespace

extern "C" {

mrg_status mrg_seed_from_master(uint64_t master_seed, uint32_t out6[6])
{
    if (!out6) return set_error(MRG_EINVAL, "null output");
    mrg::expand_seed(master_seed, out6);
    return MRG_OK;
}

mrg_status mrg_jump_matrix(int component, const uint64_t h_exp[3], uint32_t out9[9])
{
    if (!h_exp || !out9) return set_error(MRG_EINVAL, "null argument");
    if (component != 0 && component != 1) return set_error(MRG_EINVAL, "component must be 0 or 1");
    const Mat R = power(component, h_exp);
    std::memcpy(out9, R.data(), 36);
    return MRG_OK;
}

mrg_status mrg_state_check(const uint32_t state6[6])
{
    if (!state6) return set_error(MRG_EINVAL, "null state");
    if (!state_ok(state6)) return set_error(MRG_EINVAL, "invalid MRG32k3a state");
    return MRG_OK;
}

mrg_status mrg_streamset_create(mrg_streamset *out, uint64_t n_streams, uint64_t first_stream,
                                const uint32_t seed6[6], void *stream)
{
    if (!out || !seed6) return set_error(MRG_EINVAL, "null argument");
    *out = nullptr;
    if (!state_ok(seed6)) return set_error(MRG_EINVAL, "invalid seed state");
    mrg_streamset ss;
    DevCtx *ctx;
    mrg_status st = new_streamset(n_streams, first_stream, &ss, &ctx);
    if (st) return st;
    std::memcpy(ss->seed, seed6, sizeof ss->seed);
    // exponent g * 2^127 uses bits 127 .. 126 + bit_length(g): windows 31 ..
    const uint64_t g_max = first_stream + (n_streams - 1);
    const int top_bit = 126 + bit_length(g_max);  // highest set bit of g_max * 2^127
    const int w_lo = 31, w_hi = g_max ? top_bit / 4 + 1 : 31;
    mrg::InitSeed sd;
    std::memcpy(sd.w, seed6, sizeof sd.w);
    hipError_t e = mrg::launch_init(ss->d_planes, n_streams, n_streams, first_stream, sd,
                                    ctx->d_table, w_lo, w_hi, (hipStream_t)stream);
    if (e != hipSuccess) {
        (void)hipFree(ss->d_planes);
        delete ss;
        return hip_error(e, "init kernel launch");
    }
    *out = ss;
    return MRG_OK;
}

mrg_status mrg_streamset_create_seed64(mrg_streamset *out, uint64_t n_streams,
                                       uint64_t first_stream, uint64_t master_seed, void *stream)
{
    uint32_t s[6];
    mrg_status st = mrg_seed_from_master(master_seed, s);
    if (st) return st;
    return mrg_streamset_create(out, n_streams, first_stream, s, stream);
}

mrg_status mrg_streamset_create_random(mrg_streamset *out, uint64_t n_streams,
                                       uint64_t first_stream, uint64_t master_seed, void *stream)
{
    if (!out) return set_error(MRG_EINVAL, "null argument");
    *out = nullptr;
    mrg_streamset ss;
    DevCtx *ctx;
    mrg_status st = new_streamset(n_streams, first_stream, &ss, &ctx);
    if (st) return st;
    // no common base state: info reports all zeros
    hipError_t e = mrg::launch_random_init(ss->d_planes, n_streams, n_streams, first_stream,
                                           master_seed, (hipStream_t)stream);
    if (e != hipSuccess) {
        (void)hipFree(ss->d_planes);
        delete ss;
        return hip_error(e, "random init kernel launch");
    }
    *out = ss;
    return MRG_OK;
}

mrg_status mrg_streamset_create_philox(mrg_streamset *out, uint64_t n_streams,
                                       uint64_t first_stream, uint64_t key, void *stream)
{
    if (!out) return set_error(MRG_EINVAL, "null argument");
    *out = nullptr;
    mrg_streamset ss;
    DevCtx *ctx;
    mrg_status st = new_streamset(n_streams, first_stream, &ss, &ctx);
    if (st) return st;
    ss->gen = 1;
    hipError_t e = mrg::launch_philox_init(ss->d_planes, n_streams, n_streams, first_stream, key,
                                           (hipStream_t)stream);
    if (e != hipSuccess) {
        (void)hipFree(ss->d_planes);
        delete ss;
        return hip_error(e, "philox init kernel launch");
    }
    *out = ss;
    return MRG_OK;
}

mrg_status mrg_streamset_destroy(mrg_streamset ss)
{
    if (!ss) return MRG_OK;
    mrg_status st = MRG_OK;
    if (ss->d_planes) {
        int prev = -1;
        (void)hipGetDevice(&prev);
        if (prev != ss->device) (void)hipSetDevice(ss->device);
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) st = hip_error(e, "hipDeviceSynchronize before free");
        e = hipFree(ss->d_planes);
        if (e != hipSuccess && st == MRG_OK) st = hip_error(e, "hipFree(states)");
        if (ss->d_records) {
            e = hipFree(ss->d_records);
            if (e != hipSuccess && st == MRG_OK) st = hip_error(e, "hipFree(parameter records)");
        }
        if (prev != ss->device && prev >= 0) (void)hipSetDevice(prev);
    }
    delete ss;
    return st;
}

mrg_status mrg_streamset_info(mrg_streamset ss, uint64_t *n_streams, uint64_t *first_stream,
                              uint32_t seed6[6])
{
    if (!ss) return set_error(MRG_EINVAL, "null stream set");
    if (n_streams) *n_streams = ss->n;
    if (first_stream) *first_stream = ss->first;
    if (seed6) std::memcpy(seed6, ss->seed, sizeof ss->seed);
    return MRG_OK;
}

mrg_status mrg_streamset_states_ptr(mrg_streamset ss, void **d_states)
{
    if (!ss || !d_states) return set_error(MRG_EINVAL, "null argument");
    *d_states = ss->d_planes;
    return MRG_OK;
}

mrg_status mrg_streamset_tables_ptr(mrg_streamset ss, const void **d_tables)
{
    mrg_status st = check_set(ss);
    if (st) return st;
    if (!d_tables) return set_error(MRG_EINVAL, "null argument");
    DevCtx *ctx;
    if ((st = device_ctx(ss->device, &ctx))) return st;
    *d_tables = ctx->d_table;
    return MRG_OK;
}

mrg_status mrg_jump(mrg_streamset ss, uint64_t first, uint64_t count, const uint64_t *d_exp,
                    void *stream)
{
    mrg_status st = check_set(ss);
    if (st) return st;
    if ((st = check_range(ss, first, count))) return st;
    if (count == 0) return MRG_OK;
    if (!d_exp) return set_error(MRG_EINVAL, "null exponent array");
    if ((st = mrg::check_device_span(d_exp, 24 * count, ss->device, "exponent array"))) return st;
    if (ss->gen == mrg::kGenPhilox) {  // the position moves by e mod 2^64
        hipError_t e = mrg::launch_philox_jump(ss->d_planes, ss->n, first, count, d_exp, 0,
                                               (hipStream_t)stream);
        return e == hipSuccess ? MRG_OK : hip_error(e, "jump kernel launch");
    }
    if (ss->gen == mrg::kGenTinyMT) {
        const uint64_t none[3] = {0, 0, 0};
        hipError_t e = mrg::launch_tmt_jump(ss->d_planes, ss->n, first, count, d_exp, none,
                                            ss->d_records, ss->q0, (hipStream_t)stream);
        return e == hipSuccess ? MRG_OK : hip_error(e, "jump kernel launch");
    }
    DevCtx *ctx;
    if ((st = device_ctx(ss->device, &ctx))) return st;
    hipError_t e = mrg::launch_jump(ss->d_planes, ss->n, first, count, d_exp, ctx->d_table,
                                    (hipStream_t)stream);
    return e == hipSuccess ? MRG_OK : hip_error(e, "jump kernel launch");
}

mrg_status mrg_jump_uniform(mrg_streamset ss, uint64_t first, uint64_t count,
                            const uint64_t h_exp[3], void *stream)
{
    mrg_status st = check_set(ss);
    if (st) return st;
    if ((st = check_range(ss, first, count))) return st;
    if (!h_exp) return set_error(MRG_EINVAL, "null exponent");
    if (count == 0) return MRG_OK;
    if (ss->gen == mrg::kGenPhilox) {
        hipError_t e = mrg::launch_philox_jump(ss->d_planes, ss->n, first, count, nullptr,
                                               h_exp[0], (hipStream_t)stream);
        return e == hipSuccess ? MRG_OK : hip_error(e, "jump kernel launch");
    }
    if (ss->gen == mrg::kGenTinyMT) {
        hipError_t e = mrg::launch_tmt_jump(ss->d_planes, ss->n, first, count, nullptr, h_exp,
                                            ss->d_records, ss->q0, (hipStream_t)stream);
        return e == hipSuccess ? MRG_OK : hip_error(e, "jump kernel launch");
    }
    hipError_t e = mrg::launch_jump_uniform(ss->d_planes, ss->n, first, count,
                                            jump_matrices(h_exp), (hipStream_t)stream);
    return e == hipSuccess ? MRG_OK : hip_error(e, "jump kernel launch");
}

mrg_status mrg_jump_substreams(mrg_streamset ss, uint64_t first, uint64_t count, uint64_t k,
                               void *stream)
{
    if (ss && ss->gen != mrg::kGenMRG)
        return set_error(MRG_EINVAL, "substreams are defined for MRG32k3a stream sets only");
    // k * 2^76 = (k << 12) * 2^64 + (k >> 52) * 2^128
    const uint64_t e[3] = {0, k << 12, k >> 52};
    return mrg_jump_uniform(ss, first, count, e, stream);
}

mrg_status mrg_fill(mrg_streamset ss, uint64_t first, uint64_t count, uint64_t n_per_stream,
                    mrg_dtype dtype, mrg_layout layout, void *d_out, void *stream)
{
    mrg_status st = check_set(ss);
    if (st) return st;
    if ((st = check_range(ss, first, count))) return st;
    if (dtype != MRG_U32 && dtype != MRG_F32 && dtype != MRG_F64)
        return set_error(MRG_EINVAL, "unknown dtype %d", (int)dtype);
    if (layout != MRG_STREAM_MAJOR && layout != MRG_INTERLEAVED)
        return set_error(MRG_EINVAL, "unknown layout %d", (int)layout);
    if (count == 0 || n_per_stream == 0) return MRG_OK;
    if (!d_out) return set_error(MRG_EINVAL, "null output");
    const uint64_t es = dtype == MRG_F64 ? 8 : 4;
    if ((uintptr_t)d_out % es) return set_error(MRG_EINVAL, "output not aligned to its element size");
    if (n_per_stream > UINT64_MAX / es / count)
        return set_error(MRG_ERANGE, "output size overflows 64 bits");
    if ((st = mrg::check_device_span(d_out, count * n_per_stream * es, ss->device, "output")))
        return st;
    if (ss->gen == mrg::kGenPhilox) {
        hipError_t e = mrg::launch_philox_fill(ss->d_planes, ss->n, first, count, n_per_stream,
                                               (int)dtype, (int)layout, d_out, (hipStream_t)stream);
        if (e == hipSuccess)
            e = mrg::launch_philox_jump(ss->d_planes, ss->n, first, count, nullptr, n_per_stream,
                                        (hipStream_t)stream);
        return e == hipSuccess ? MRG_OK : hip_error(e, "philox fill kernel launch");
    }
    const mrg::FillTuning tune = tuning();
    if (ss->gen == mrg::kGenTinyMT) {
        hipError_t e = mrg::launch_tmt_fill(ss->d_planes, ss->n, first, count, n_per_stream,
                                            (int)dtype, (int)layout, d_out, ss->d_records, ss->q0,
                                            tune.tile_bytes, (hipStream_t)stream);
        return e == hipSuccess ? MRG_OK : hip_error(e, "tinymt fill kernel launch");
    }
    mrg::FillLaunch fl;
    if (layout == MRG_STREAM_MAJOR) {
        // wave per stream when a stream fills at least one chunk of 64 lanes x
        // 128 bytes (or when forced; see below for rows under 16 KiB); lane per
        // stream for short streams
        const uint64_t min_chunk = 64 * (128 / es);
        const bool coop = tune.strategy == 2 || (tune.strategy == 0 && n_per_stream >= min_chunk);
        if (coop) {
            DevCtx *ctx;
            if ((st = device_ctx(ss->device, &ctx))) return st;
            // GL lanes per stream, 64/GL streams per wave; each lane takes
            // 64/GL or 2*64/GL pieces of 128 bytes per chunk (a chunk is then
            // 64 or 128 lines), whichever generates fewer values past the end
            // of a row (the longer chunk on a tie).  A row's line-aligned
            // part is n values, or about n - tv/2 when rows start anywhere.
            // automatic: 16 lanes for rows under 64 KiB, else 64 (measured
            // faster for rows of 64 KiB and more)
            const int GL = tune.coop_lanes ? tune.coop_lanes : n_per_stream * es >= 65536 ? 64 : 16;
            const uint64_t tv = 128 / es;
            const uint64_t nh_min = 64 / GL, nh_max = 2 * nh_min;
            const bool rows_aligned = (uintptr_t)d_out % 128 == 0 && (n_per_stream * es) % 128 == 0;
            const uint64_t body = rows_aligned || n_per_stream <= tv ? n_per_stream : n_per_stream - tv / 2;
            const uint64_t ch_min = (uint64_t)GL * nh_min * tv, ch_max = 2 * ch_min;
            const uint64_t gen_min = (body + ch_min - 1) / ch_min * ch_min;
            const uint64_t gen_max = (body + ch_max - 1) / ch_max * ch_max;
            const uint64_t nh = gen_max <= gen_min ? nh_max : nh_min;
            const int L = (int)(nh * tv);
            if (L % 16 || L < 16 || L > 512) return set_error(MRG_EINVAL, "no lane table for L = %d", L);
            fl.kernel = 1;
            fl.L = L;
            fl.lanes = GL;
            fl.lane_tab = ctx->d_lane_tab + mrg::lane_table(L) * 64 * 18;
            fl.tabs = ctx->d_lane_tab;
            fl.table = ctx->d_table;
            // resident workgroups stride over the stream groups, or one per group
            const uint64_t groups = (count + (64 / GL) - 1) / (64 / GL);
            const uint64_t cap = tune.coop_wgs_per_cu ? (uint64_t)ctx->cus * tune.coop_wgs_per_cu
                                                      : ((uint64_t)1 << 31) - 1;
            fl.grid = (unsigned)(groups < cap ? groups : cap);
            fl.order = tune.coop_order;
            // the bulk case: rows on lines, whole chunks, a group's rows
            // addressable with 32-bit offsets
            fl.whole = rows_aligned && n_per_stream % ((uint64_t)GL * L) == 0 &&
                       (uint64_t)(64 / GL) * n_per_stream * es < ((uint64_t)1 << 32);
            // automatic choice: a row under 16 KiB that is not whole chunks on
            // lines is one cut chunk for this writer (values drawn past the
            // row's end, one piece per flush), and with enough streams to fill
            // the chip one lane each (2048 waves of 64) the lane-per-stream
            // writer is the faster one (uint32 rows of 3000: 4.0-4.5 against
            // 3.4 TB/s; of 4000: 4.2-4.4 against 3.6-3.7; from 4500 values
            // this writer leads, 4.7-4.8 against 4.0-4.5).  With fewer streams
            // this writer's 16 lanes per stream keep the launch short.
            if (tune.strategy == 0 && !fl.whole && n_per_stream * es < 16 * 1024 &&
                count >= ((uint64_t)64 << 11))
                fl = mrg::FillLaunch();
        }
    }
    hipError_t e = mrg::launch_fill(ss->d_planes, ss->n, first, count, n_per_stream, (int)dtype,
                                    (int)layout, d_out, fl, tune, (hipStream_t)stream);
    return e == hipSuccess ? MRG_OK : hip_error(e, "fill kernel launch");
}

mrg_status mrg_fill_leapfrog(mrg_streamset ss, uint64_t s, uint64_t players,
                             uint64_t per_player, mrg_dtype dtype, mrg_layout layout,
                             void *d_out, void *stream)
{
    mrg_status st = check_set(ss);
    if (st) return st;
    if ((st = check_range(ss, s, 1))) return st;
    if (dtype != MRG_U32 && dtype != MRG_F32 && dtype != MRG_F64)
        return set_error(MRG_EINVAL, "unknown dtype %d", (int)dtype);
    if (layout != MRG_STREAM_MAJOR && layout != MRG_INTERLEAVED)
        return set_error(MRG_EINVAL, "unknown layout %d", (int)layout);
    if (ss->gen != mrg::kGenMRG)
        return set_error(MRG_EINVAL, "leapfrog is defined for MRG32k3a stream sets only");
    if (players == 0 || per_player == 0) return MRG_OK;
    if (!d_out) return set_error(MRG_EINVAL, "null output");
    const uint64_t es = dtype == MRG_F64 ? 8 : 4;
    if ((uintptr_t)d_out % es) return set_error(MRG_EINVAL, "output not aligned to its element size");
    if (players > UINT64_MAX / per_player || players * per_player > UINT64_MAX / es)
        return set_error(MRG_ERANGE, "players * per_player * element size overflows 64 bits");
    const uint64_t N = players * per_player;
    if ((st = mrg::check_device_span(d_out, N * es, ss->device, "output"))) return st;
    DevCtx *ctx;
    if ((st = device_ctx(ss->device, &ctx))) return st;
    const mrg::FillTuning tune = tuning();
    mrg::PartitionLaunch pl;
    pl.table = ctx->d_table;
    const uint64_t slots = (uint64_t)ctx->cus * 16;  // resident one-wave workgroups
    // with one player or one card per player both layouts are the stream in order
    if (layout == MRG_INTERLEAVED || players == 1 || per_player == 1) {
        // the stream's outputs in order: blocks of 16-256 KiB (at least 4096
        // of them when the output allows), each a whole number of 128-line
        // chunks, one 64-lane wave per block
        const uint64_t tv = 128 / es;
        uint64_t bb = 16384;
        while (bb < 262144 && N * es / (2 * bb) >= 4096) bb *= 2;
        pl.kind = 0;
        pl.B = bb / es;
        pl.nfull = N / pl.B;
        pl.rem = N % pl.B;
        const bool one_chunk = N < 128 * tv;  // short: 64-line chunks
        pl.L = (int)(one_chunk ? tv : 2 * tv);
        pl.lane_tab = ctx->d_lane_tab + mrg::lane_table(pl.L) * 64 * 18;
        pl.tabs = ctx->d_lane_tab;
        const uint64_t blocks = pl.nfull + (pl.rem ? 1 : 0);
        pl.grid = (unsigned)(blocks < ((uint64_t)1 << 31) - 1 ? blocks : ((uint64_t)1 << 31) - 1);
    } else {
        // each player's cards in a row: items of KB = min(K, 64) card columns
        // x T players (R = 64 / KB lanes per column, Ts = T / R players
        // each), T chosen for about 4 items per resident workgroup (at least
        // 256 players per lane)
        mrg::LeapArgs &A = pl.leap;
        pl.kind = 1;
        A.P = players;
        A.K = per_player;
        A.KB = (int)(per_player < 64 ? per_player : 64);
        A.R = 64 / A.KB;
        const uint64_t nkb = (per_player + A.KB - 1) / A.KB;
        const uint64_t target = 4 * slots;
        uint64_t Ts = (players + A.R - 1) / A.R;
        if (nkb < target) {
            const uint64_t segs = (target + nkb - 1) / nkb;
            Ts = (players + segs * A.R - 1) / (segs * A.R);
            if (Ts < 256) Ts = 256;
        }
        const uint64_t ts_max = (players + A.R - 1) / A.R;
        if (Ts > ts_max) Ts = ts_max;
        A.Ts = Ts;
        A.T = Ts * A.R;
        A.nseg = (players + A.T - 1) / A.T;
        A.items = nkb * A.nseg;
        pl.grid = (unsigned)(A.items < slots ? A.items : slots);
        // 63 * players and T - Ts as 192-bit exponents
        const unsigned __int128 e63 = (unsigned __int128)players * 63u;
        const uint64_t ew[3] = {(uint64_t)e63, (uint64_t)(e63 >> 64), 0};
        A.J63 = jump_matrices(ew);
        const uint64_t es_[3] = {A.T - A.Ts, 0, 0};
        A.Jseg = jump_matrices(es_);
    }
    hipError_t e = mrg::launch_partition(ss->d_planes, ss->n, s, (int)dtype, pl, d_out,
                                         tune.engine, (hipStream_t)stream);
    if (e != hipSuccess) return hip_error(e, "leapfrog kernel launch");
    // the stream moves past the N outputs dealt
    const uint64_t en[3] = {N, 0, 0};
    e = mrg::launch_jump_uniform(ss->d_planes, ss->n, s, 1, jump_matrices(en), (hipStream_t)stream);
    return e == hipSuccess ? MRG_OK : hip_error(e, "jump kernel launch");
}

mrg_status mrg_get_states(mrg_streamset ss, uint64_t first, uint64_t count, uint32_t *h_out,
                          void *stream)
{
    mrg_status st = check_set(ss);
    if (st) return st;
    if ((st = check_range(ss, first, count))) return st;
    if (count == 0) return MRG_OK;
    if (!h_out) return set_error(MRG_EINVAL, "null output");
    std::vector<uint32_t> tmp(6 * count);
    for (int c = 0; c < 6; ++c) {
        hipError_t e = hipMemcpyAsync(tmp.data() + c * count, ss->d_planes + c * ss->n + first,
                                      count * 4, hipMemcpyDeviceToHost, (hipStream_t)stream);
        if (e != hipSuccess) return hip_error(e, "hipMemcpyAsync(states)");
    }
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_error(e, "hipStreamSynchronize");
    for (uint64_t i = 0; i < count; ++i)
        for (int c = 0; c < 6; ++c) h_out[6 * i + c] = tmp[c * count + i];
    return MRG_OK;
}

mrg_status mrg_set_states(mrg_streamset ss, uint64_t first, uint64_t count, const uint32_t *h_in,
                          void *stream)
{
    mrg_status st = check_set(ss);
    if (st) return st;
    if ((st = check_range(ss, first, count))) return st;
    if (count == 0) return MRG_OK;
    if (!h_in) return set_error(MRG_EINVAL, "null input");
    for (uint64_t i = 0; ss->gen == mrg::kGenMRG && i < count; ++i)  // any 6 words are a Philox state
        if (!state_ok(h_in + 6 * i))
            return set_error(MRG_EINVAL, "state %llu is not a valid MRG32k3a state",
                        (unsigned long long)i);
    for (uint64_t i = 0; ss->gen == mrg::kGenTinyMT && i < count; ++i) {
        // a TinyMT state: nonzero 127-bit part, a parameter set of this set
        // (the one its stream was created with), word 5 zero
        const uint32_t *w = h_in + 6 * i;
        const uint64_t q_want = (ss->first + first + i) / ss->per_param;
        if (((w[0] & 0x7fffffffu) | w[1] | w[2] | w[3]) == 0u || w[4] != q_want || w[5] != 0u)
            return set_error(MRG_EINVAL, "state %llu is not a TinyMT32 state of its stream "
                             "(nonzero state, parameter set %llu, last word 0)",
                             (unsigned long long)i, (unsigned long long)q_want);
    }
    std::vector<uint32_t> tmp(6 * count);
    for (uint64_t i = 0; i < count; ++i)
        for (int c = 0; c < 6; ++c) tmp[c * count + i] = h_in[6 * i + c];
    for (int c = 0; c < 6; ++c) {
        hipError_t e = hipMemcpyAsync(ss->d_planes + c * ss->n + first, tmp.data() + c * count,
                                      count * 4, hipMemcpyHostToDevice, (hipStream_t)stream);
        if (e != hipSuccess) return hip_error(e, "hipMemcpyAsync(states)");
    }
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    return e == hipSuccess ? MRG_OK : hip_error(e, "hipStreamSynchronize");
}

mrg_status mrg_config_set(const char *key, int64_t value)
{
    if (!key) return set_error(MRG_EINVAL, "null key");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!std::strcmp(key, "engine")) {
        if (value != 0 && value != 1) return set_error(MRG_EINVAL, "engine must be 0 or 1");
        g_tune.engine = (int)value;
    } else if (!std::strcmp(key, "coop_order")) {
        if (value != 0 && value != 1) return set_error(MRG_EINVAL, "coop_order must be 0 or 1");
        g_tune.coop_order = (int)value;
    } else if (!std::strcmp(key, "coop_wgs_per_cu")) {
        if (value < 0 || value > 1024) return set_error(MRG_EINVAL, "coop_wgs_per_cu must be in [0, 1024]");
        g_tune.coop_wgs_per_cu = (int)value;
    } else if (!std::strcmp(key, "coop_lanes")) {
        if (value != 64 && value != 32 && value != 16 && value != 8 && value != 0)
            return set_error(MRG_EINVAL, "coop_lanes must be 0, 64, 32, 16 or 8");
        g_tune.coop_lanes = (int)value;
    } else if (!std::strcmp(key, "strategy")) {
        if (value < 0 || value > 2) return set_error(MRG_EINVAL, "strategy must be 0, 1 or 2");
        g_tune.strategy = (int)value;
    } else if (!std::strcmp(key, "tile_bytes")) {
        if (value != 0 && value != 128 && value != 256)
            return set_error(MRG_EINVAL, "tile_bytes must be 0 (automatic), 128 or 256");
        g_tune.tile_bytes = (int)value;
    } else {
        return set_error(MRG_EINVAL, "unknown key '%s'", key);
    }
    return MRG_OK;
}

mrg_status mrg_config_get(const char *key, int64_t *value)
{
    if (!key || !value) return set_error(MRG_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!std::strcmp(key, "engine")) *value = g_tune.engine;
    else if (!std::strcmp(key, "tile_bytes")) *value = g_tune.tile_bytes;
    else if (!std::strcmp(key, "strategy")) *value = g_tune.strategy;
    else if (!std::strcmp(key, "coop_wgs_per_cu")) *value = g_tune.coop_wgs_per_cu;
    else if (!std::strcmp(key, "coop_order")) *value = g_tune.coop_order;
    else if (!std::strcmp(key, "coop_lanes")) *value = g_tune.coop_lanes;
    else return set_error(MRG_EINVAL, "unknown key '%s'", key);
    return MRG_OK;
}

const char *mrg_status_string(mrg_status s)
{
    switch (s) {
    case MRG_OK: return "MRG_OK";
    case MRG_EINVAL: return "MRG_EINVAL: invalid argument";
    case MRG_ENOMEM: return "MRG_ENOMEM: allocation failed";
    case MRG_EHIP: return "MRG_EHIP: HIP runtime error";
    case MRG_ERANGE: return "MRG_ERANGE: out of range";
    case MRG_ENODEV: return "MRG_ENODEV: no HIP device";
    case MRG_EBUSY: return "MRG_EBUSY: waiting on memory or time";
    default: return "unknown mrg_status";
    }
}

const char *mrg_last_error(void) { return g_last_error.c_str(); }

mrg_status mrg_write_probe(void *d_out, uint64_t bytes, int32_t pattern, void *stream)
{
    if (pattern < 0 || pattern > 3) return set_error(MRG_EINVAL, "unknown probe pattern %d", pattern);
    if (!d_out) return set_error(MRG_EINVAL, "null output");
    const uint64_t unit = pattern == 0 ? 16 : 65536, align = pattern == 0 ? 16 : 128;
    if (bytes % unit) return set_error(MRG_EINVAL, "probe size must be a multiple of %llu bytes",
                                       (unsigned long long)unit);
    if ((uintptr_t)d_out % align) return set_error(MRG_EINVAL, "probe output must be %llu-byte aligned",
                                                   (unsigned long long)align);
    if (!bytes) return MRG_OK;
    int dev;
    mrg_status st = current_device(&dev);
    if (st) return st;
    if ((st = mrg::check_device_span(d_out, bytes, dev, "probe output"))) return st;
    hipError_t e = mrg::launch_write_probe(d_out, bytes, pattern, (hipStream_t)stream);
    return e == hipSuccess ? MRG_OK : hip_error(e, "probe launch");
}

int32_t mrg_version(void) { return 100; }

}  // extern "C"
