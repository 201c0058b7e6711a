// qai_api.hip -- the C ABI of libqai: argument validation, workspace layout,
// stream-ordered dispatch of the post-pass, status and error reporting,
// stage timing and the bandwidth probe.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "qai.h"
#include "qai_device.h"
#include "qai_kernels.h"

namespace qai {
namespace api {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int fail_hip(hipError_t e, const char* what)
{
    return fail(QAI_EHIP, "%s: %s", what, hipGetErrorString(e));
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

int check_dims(const int64_t dims[3], int64_t* n)
{
    if (!dims)
        return fail(QAI_EINVAL, "dims is NULL");
    for (int a = 0; a < 3; ++a)
        if (dims[a] < 1 || dims[a] > QAI_MAX_EXTENT)
            return fail(QAI_EDIMS, "extent %d = %lld outside [1, %d]", a, (long long)dims[a], QAI_MAX_EXTENT);
    *n = dims[0] * dims[1] * dims[2];
    return QAI_OK;
}

int check_eb(float eb)
{
    if (!(eb > 0.0f) || !isfinite(eb))
        return fail(QAI_EINVAL, "error bound must be finite and > 0 (got %g)", (double)eb);
    const float two = 2.0f * eb, inv = 1.0f / two;
    if (!isfinite(two) || !isfinite(inv) || !(inv > 0.0f))
        return fail(QAI_EINVAL, "error bound %g out of the representable range", (double)eb);
    return QAI_OK;
}

int check_params(const qai_params* p, qai_params* out)
{
    qai_params d = {0.9f, 1.0f, 0u};
    if (p)
        d = *p;
    if (!isfinite(d.eta))
        return fail(QAI_EINVAL, "eta must be finite");
    if (!isfinite(d.power) || !(d.power > 0.0f))
        return fail(QAI_EINVAL, "power must be finite and > 0");
    if (d.flags != 0u)
        return fail(QAI_EINVAL, "params.flags is reserved and must be 0");
    *out = d;
    return QAI_OK;
}

} // namespace api
} // namespace qai

using namespace qai::api;

namespace {

// ---- stage timing
struct StageRec {
    const char* name;
    hipEvent_t a, b;
};
std::mutex g_prof_mu;
std::mutex g_tune_mu;
bool g_tune_set = false;
bool g_tune_user = false; // set by qai_tuning_set with a setting (not NULL)
qai::Tuning g_tune;

qai::Tuning current_tuning()
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_tune_set) {
        qai::default_tuning(g_tune);
        g_tune_set = true;
    }
    return g_tune;
}
bool g_prof_on = false;
thread_local int g_prof_suppress = 0; // stage timing paused (graph capture)
std::vector<StageRec> g_pending;
std::vector<std::pair<const char*, double>> g_acc;
thread_local hipEvent_t g_cur_a = nullptr;
thread_local const char* g_cur_name = nullptr;

} // namespace

namespace qai {

int kernel_block_limit(const void* fn)
{
    static std::mutex mu;
    static std::vector<std::pair<const void*, int>> cache;
    std::lock_guard<std::mutex> lk(mu);
    for (const auto& kv : cache)
        if (kv.first == fn)
            return kv.second;
    hipFuncAttributes at;
    if (hipFuncGetAttributes(&at, fn) != hipSuccess)
        return 0;
    cache.push_back({fn, at.maxThreadsPerBlock});
    return at.maxThreadsPerBlock;
}

void prof_begin(const char* name, hipStream_t s)
{
    if (!g_prof_on || g_prof_suppress)
        return;
    hipEvent_t a;
    if (hipEventCreate(&a) != hipSuccess)
        return;
    (void)hipEventRecord(a, s);
    g_cur_a = a;
    g_cur_name = name;
}

void prof_end(hipStream_t s)
{
    if (!g_prof_on || g_prof_suppress || !g_cur_a)
        return;
    hipEvent_t b;
    if (hipEventCreate(&b) != hipSuccess)
        return;
    (void)hipEventRecord(b, s);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_pending.push_back({g_cur_name, g_cur_a, b});
    g_cur_a = nullptr;
}

namespace api {

Tuning tuning_now() { return current_tuning(); }

// The setting a plain call on dims runs with: a shape's autotuned entry while
// the process-wide setting is the built-in default, else that setting.
Tuning tuning_for(const int64_t dims[3])
{
    bool user;
    Tuning t;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        if (!g_tune_set) {
            default_tuning(g_tune);
            g_tune_set = true;
        }
        t = g_tune;
        user = g_tune_user;
    }
    Tuning c;
    if (!user && cache_lookup(dims, c))
        return c;
    return t;
}

void prof_suppress(bool on) { g_prof_suppress += on ? 1 : -1; }

// k-th region after the header; cap = word_capacity of the field
uint32_t* word_buffer(void* ws, int64_t cap, int k)
{
    return (uint32_t*)((unsigned char*)ws + kHeaderBytes + (size_t)k * align256((size_t)cap * 4));
}

// the field's extents must be set in p
void ws_buffers(void* ws, Plan1& p)
{
    const int64_t cap = qai::word_capacity(p.nz, p.ny, p.nx);
    p.status = (uint32_t*)ws;
    p.bufA = word_buffer(ws, cap, 0);
    p.bufB = word_buffer(ws, cap, 1);
    p.bufC = word_buffer(ws, cap, 2);
    p.flags = (uint64_t*)word_buffer(ws, cap, 3);
}

void clear_error() { g_err.clear(); }

int abi_to_tuning(const qai_tuning* in, Tuning& t)
{
    default_tuning(t);
    for (int k = 0; k < 2; ++k) {
        if (in->edt1_algo[k] < -1 || in->edt1_algo[k] > 5 || in->edt1_algo[k] == 3 || in->edt2_algo[k] < -1 ||
            in->edt2_algo[k] > 5)
            return fail(QAI_EINVAL, "algorithm choice: -1 (auto), 0, 1, 2, 4 or 5 for the first EDT, -1..5 for the second");
        if (in->tile_log2[k] < -1 || in->tile_log2[k] > 6)
            return fail(QAI_EINVAL, "tile_log2 must be in [-1, 6]");
    }
    for (int r : {in->edt1_ring, in->edt2_ring})
        if (r != 16 && r != 32 && r != 64)
            return fail(QAI_EINVAL, "ring sizes must be 16, 32 or 64");
    if (in->seed_rows < -1 || in->seed_rows > 8 || in->seed_planes < 1 || in->seed_planes > 4096)
        return fail(QAI_EINVAL, "seed_rows must be in [-1, 8] and seed_planes in [1, 4096]");
    if (in->window_threads < 64 || in->window_threads > 1024 || in->window_threads % 64)
        return fail(QAI_EINVAL, "window_threads must be a multiple of 64 in [64, 1024]");
    if (in->force_wide != 0 && in->force_wide != 1)
        return fail(QAI_EINVAL, "force_wide must be 0 or 1");
    for (int a = 1; a <= 2; ++a) {
        t.edt1_algo[a] = in->edt1_algo[a - 1];
        t.env_algo[a] = in->edt2_algo[a - 1];
        t.edt1_cap[a] = in->edt1_ring;
        t.stream_cap[a] = in->edt2_ring;
        t.env_tx_log2[a] = in->tile_log2[a - 1];
    }
    t.seed_ty = in->seed_rows;
    t.seed_tz = in->seed_planes;
    t.env_threads = in->window_threads;
    t.force_wide = in->force_wide;
    return QAI_OK;
}

int tuning_to_abi(const Tuning& t, qai_tuning* out)
{
    out->edt1_algo[0] = t.edt1_algo[1];
    out->edt1_algo[1] = t.edt1_algo[2];
    out->edt2_algo[0] = t.env_algo[1];
    out->edt2_algo[1] = t.env_algo[2];
    out->edt1_ring = t.edt1_cap[1];
    out->edt2_ring = t.stream_cap[1];
    out->tile_log2[0] = t.env_tx_log2[1];
    out->tile_log2[1] = t.env_tx_log2[2];
    out->seed_rows = t.seed_ty;
    out->seed_planes = t.seed_tz;
    out->window_threads = t.env_threads;
    out->force_wide = t.force_wide;
    return QAI_OK;
}

} // namespace api

hipError_t launch_backward(const float* g, const uint32_t* w1, const uint32_t* w2, int64_t n, float eb, float eta,
                           float power, double* partial, float* out, hipStream_t s);
void final_buffers(int64_t nz, int64_t ny, int64_t nx, int& w1, int& w2);

} // namespace qai

namespace {

constexpr size_t kPartialOffset = 256; // FP64 partial sums of the adjoint reduction


// side: run the streaming part of step E on the device's side stream
// alongside the second EDT's y pass (qai::Aux), unless stream is being
// captured; the allocation-free entry point keeps every launch on stream
int plain_checked(const float* field, const int64_t dims[3], float eb, const qai_params* params, void* ws,
                  size_t ws_bytes, float* out, const qai_taps* taps, void* stream, bool side)
{
    int64_t n;
    int rc = check_dims(dims, &n);
    if (rc)
        return rc;
    if (!field || !out)
        return fail(QAI_EINVAL, "field and out must be device pointers");
    if ((rc = check_eb(eb)))
        return rc;
    qai_params p;
    if ((rc = check_params(params, &p)))
        return rc;
    const size_t need = qai_workspace_bytes(dims);
    if (!ws || ws_bytes < need)
        return fail(QAI_ENOWS, "workspace of %zu bytes needed, %zu given", need, ws ? ws_bytes : (size_t)0);
    if (((uintptr_t)ws & 255u) != 0)
        return fail(QAI_ENOWS, "workspace must be 256-byte aligned");
    const float* fe = field + n;
    if (out != field && ((out > field && out < fe) || (field > out && field < out + n)))
        return fail(QAI_EINVAL, "out partly overlaps field");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fail(QAI_ENODEV, "no usable GPU: %s", hipGetErrorString(e));

    qai::Plan1 pl = {};
    pl.xq = field;
    pl.out = out;
    pl.nz = dims[0];
    pl.ny = dims[1];
    pl.nx = dims[2];
    pl.eb = eb;
    pl.eta = p.eta;
    pl.power = p.power;
    ws_buffers(ws, pl);
    if (taps)
        pl.taps = *taps;
    const qai::Tuning t = tuning_for(dims);
    std::unique_lock<std::mutex> lk;
    if (side && !qai::stream_capturing((hipStream_t)stream)) {
        if ((e = qai::aux_for(dev, pl.aux)) != hipSuccess)
            return fail_hip(e, "side stream");
        lk = std::unique_lock<std::mutex>(pl.aux->mu);
    }
    e = qai::run_plain(pl, t, (hipStream_t)stream);
    if (e != hipSuccess)
        return fail_hip(e, "kernel launch");
    return QAI_OK;
}

__global__ void k_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n16)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ void k_copy_tail(const uint32_t* src, uint32_t* dst, size_t from, size_t n)
{
    size_t i = from + (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        dst[i] = src[i];
}

// Fixed device scratch of the allocation-free entry point: the workspace of
// qai_mitigate_noalloc.  Every GPU the library runs on holds its own copy
// until the process ends.  In host code the name stands for no device
// address; the address is taken once per device with hipGetSymbolAddress.
__device__ __align__(256) unsigned char scratch[QAI_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch (looked up on the first
// call on that device, with that device current).
int scratch_on_current_device(void** ptr)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fail(QAI_ENODEV, "no usable GPU: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(QAI_ENODEV, "device ordinal %d beyond the %d the library tracks", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return fail_hip(e, "hipGetSymbolAddress(scratch)");
        if (!p || ((uintptr_t)p & 255u) != 0)
            return fail(QAI_EHIP, "scratch symbol has no 256-byte aligned device address");
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return QAI_OK;
}

} // namespace

extern "C" {

size_t qai_workspace_bytes(const int64_t dims[3])
{
    int64_t n;
    if (!dims)
        return 0;
    for (int a = 0; a < 3; ++a)
        if (dims[a] < 1 || dims[a] > QAI_MAX_EXTENT)
            return 0;
    n = dims[0] * dims[1] * dims[2];
    // three word buffers, then the fused final pass's flag words
    const int64_t cap = qai::word_capacity(dims[0], dims[1], dims[2]);
    return kHeaderBytes + 3 * align256((size_t)cap * 4) + align256(qai::flag_bytes(n));
}

int qai_mitigate_ex(const float* field, const int64_t dims[3], float eb, const qai_params* params, void* ws,
                    size_t ws_bytes, float* out, const qai_taps* taps, void* stream)
{
    g_err.clear();
    return plain_checked(field, dims, eb, params, ws, ws_bytes, out, taps, stream, true);
}

int qai_mitigate(const float* field, const int64_t dims[3], float eb, float* out, void* stream)
{
    g_err.clear();
    int64_t n;
    int rc = check_dims(dims, &n);
    if (rc)
        return rc;
    if (!field || !out)
        return fail(QAI_EINVAL, "field and out must be device pointers");
    if ((rc = check_eb(eb)))
        return rc;
    const size_t need = qai_workspace_bytes(dims);
    void* ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, need, (hipStream_t)stream);
    if (e != hipSuccess)
        return fail_hip(e, "hipMallocAsync");
    rc = plain_checked(field, dims, eb, nullptr, ws, need, out, nullptr, stream, true);
    e = hipFreeAsync(ws, (hipStream_t)stream);
    if (rc == QAI_OK && e != hipSuccess)
        return fail_hip(e, "hipFreeAsync");
    return rc;
}

int qai_mitigate_noalloc(const float* field, const int64_t dims[3], float eb, const qai_params* params, float* out,
                         void* stream)
{
    g_err.clear();
    int64_t n;
    int rc = check_dims(dims, &n);
    if (rc)
        return rc;
    const size_t need = qai_workspace_bytes(dims);
    if (need > (size_t)QAI_NOALLOC_SCRATCH_BYTES)
        return fail(QAI_ENOWS, "field needs %zu bytes of workspace; the fixed scratch holds %zu", need,
                    (size_t)QAI_NOALLOC_SCRATCH_BYTES);
    void* ws = nullptr;
    if ((rc = scratch_on_current_device(&ws)))
        return rc;
    return plain_checked(field, dims, eb, params, ws, (size_t)QAI_NOALLOC_SCRATCH_BYTES, out, nullptr, stream, false);
}

int qai_device_status(const void* ws, void* stream, uint32_t* flags)
{
    g_err.clear();
    if (!ws || !flags)
        return fail(QAI_EINVAL, "ws and flags must not be NULL");
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess)
        return fail_hip(e, "hipStreamSynchronize");
    e = hipMemcpy(flags, ws, sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return fail_hip(e, "hipMemcpy");
    return QAI_OK;
}

const char* qai_last_error(void) { return g_err.c_str(); }

int qai_backward(const float* grad_out, void* ws_saved, size_t ws_bytes, const int64_t dims[3], float eb,
                 const qai_params* params, float* grad_params, void* stream)
{
    g_err.clear();
    int64_t n;
    int rc = check_dims(dims, &n);
    if (rc)
        return rc;
    if (!grad_out || !grad_params)
        return fail(QAI_EINVAL, "grad_out and grad_params must be device pointers");
    if ((rc = check_eb(eb)))
        return rc;
    qai_params p;
    if ((rc = check_params(params, &p)))
        return rc;
    const size_t need = qai_workspace_bytes(dims);
    if (!ws_saved || ws_bytes < need)
        return fail(QAI_ENOWS, "workspace of %zu bytes needed, %zu given", need, ws_saved ? ws_bytes : (size_t)0);
    int k1, k2;
    qai::final_buffers(dims[0], dims[1], dims[2], k1, k2);
    const int64_t cap = qai::word_capacity(dims[0], dims[1], dims[2]);
    const uint32_t* w1 = word_buffer(ws_saved, cap, k1);
    const uint32_t* w2 = word_buffer(ws_saved, cap, k2);
    hipError_t e = qai::launch_backward(grad_out, w1, w2, n, eb, p.eta, p.power,
                                        (double*)((unsigned char*)ws_saved + kPartialOffset), grad_params,
                                        (hipStream_t)stream);
    return e == hipSuccess ? QAI_OK : fail_hip(e, "backward launch");
}

int qai_copy_probe(const void* src, void* dst, size_t n_words, void* stream)
{
    g_err.clear();
    if (!src || !dst)
        return fail(QAI_EINVAL, "src and dst must not be NULL");
    if (n_words == 0)
        return QAI_OK;
    const size_t n16 = ((((uintptr_t)src | (uintptr_t)dst) & 15u) == 0) ? n_words / 4 : 0;
    if (n16) {
        size_t blocks = (n16 + 255) / 256;
        if (blocks > 8192)
            blocks = 8192;
        const hipError_t e = qai::launch_checked(k_copy, dim3((uint32_t)blocks), dim3(256), 0, (hipStream_t)stream,
                                                 (const uint4*)src, (uint4*)dst, n16);
        if (e != hipSuccess)
            return fail_hip(e, "copy launch");
    }
    const size_t from = n16 * 4;
    if (from < n_words) {
        const size_t rest = n_words - from;
        const hipError_t e =
            qai::launch_checked(k_copy_tail, dim3((uint32_t)((rest + 255) / 256)), dim3(256), 0,
                                (hipStream_t)stream, (const uint32_t*)src, (uint32_t*)dst, from, n_words);
        if (e != hipSuccess)
            return fail_hip(e, "copy launch");
    }
    return QAI_OK;
}

int qai_tuning_get(qai_tuning* out)
{
    g_err.clear();
    if (!out)
        return fail(QAI_EINVAL, "tuning pointer is NULL");
    return tuning_to_abi(current_tuning(), out);
}

int qai_tuning_set(const qai_tuning* in)
{
    g_err.clear();
    qai::Tuning t;
    qai::default_tuning(t);
    if (in) {
        const int rc = abi_to_tuning(in, t);
        if (rc)
            return rc;
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune = t;
    g_tune_set = true;
    g_tune_user = in != nullptr;
    return QAI_OK;
}

int qai_profile_enable(int on)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    return QAI_OK;
}

int qai_stage_times(double* ms, const char** names, int n, int* n_stages, int reset)
{
    g_err.clear();
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto& r : g_pending) {
        hipError_t e = hipEventSynchronize(r.b);
        float t = 0.0f;
        if (e == hipSuccess)
            e = hipEventElapsedTime(&t, r.a, r.b);
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
        if (e != hipSuccess)
            continue;
        bool found = false;
        for (auto& kv : g_acc)
            if (strcmp(kv.first, r.name) == 0) {
                kv.second += t;
                found = true;
                break;
            }
        if (!found)
            g_acc.push_back({r.name, (double)t});
    }
    g_pending.clear();
    const int k = (int)g_acc.size();
    if (n_stages)
        *n_stages = k;
    for (int i = 0; i < k && i < n; ++i) {
        if (ms)
            ms[i] = g_acc[i].second;
        if (names)
            names[i] = g_acc[i].first;
    }
    if (reset)
        g_acc.clear();
    return QAI_OK;
}

} // extern "C"
