// qai_batch.hip -- batched form of the post-pass (project addition, not in
// the paper): many fields of uneven shapes run from one hipGraph.  Each field
// runs the plain pipeline's kernels on its own workspace slice; the fields are
// dealt (largest first) to a few independent branches of the graph so that
// kernels of different fields can overlap on the GPU.  Every field's result is
// bit-identical to qai_mitigate_ex on it alone, whatever the branch or tuning.
//
// With QAI_BATCH_AUTOTUNE every distinct shape runs the autotuner's setting
// for it (the cached one, or one timed now on the first field of that shape).
// All settings compute the same transform, so tuning only changes time.
#include <algorithm>
#include <map>
#include <vector>

#include "qai.h"
#include "qai_device.h"
#include "qai_kernels.h"

using namespace qai::api;

struct qai_batch_plan {
    int n = 0;
    int device = 0;
    std::vector<qai::Plan1> plans;
    std::vector<qai::Tuning> tune;
    std::vector<int> order;   // fields by decreasing size
    int branches = 1;
    hipStream_t capture = nullptr;
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> join;
    hipEvent_t fork = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

constexpr int kMaxBranches = 4; // hardware queues per process on this GPU

int64_t voxels(const int64_t d[3]) { return d[0] * d[1] * d[2]; }

void release(qai_batch_plan* p)
{
    if (!p)
        return;
    if (p->exec)
        (void)hipGraphExecDestroy(p->exec);
    if (p->graph)
        (void)hipGraphDestroy(p->graph);
    for (hipEvent_t e : p->join)
        (void)hipEventDestroy(e);
    if (p->fork)
        (void)hipEventDestroy(p->fork);
    for (hipStream_t s : p->side)
        (void)hipStreamDestroy(s);
    if (p->capture)
        (void)hipStreamDestroy(p->capture);
    delete p;
}

// Each distinct shape takes its entry of the tuning cache, or, when it has
// none, the fastest setting the tuner finds on the first field of that shape
// (then stored in the cache).
int autotune(qai_batch_plan* p, const int64_t (*dims)[3], hipStream_t s, bool each)
{
    std::map<std::vector<int64_t>, qai::Tuning> best;
    for (int i = 0; i < p->n; ++i) {
        const std::vector<int64_t> key(dims[i], dims[i] + 3);
        auto it = best.find(key);
        if (it != best.end()) {
            p->tune[i] = it->second;
            continue;
        }
        qai::Tuning pick;
        if (!qai::cache_lookup(dims[i], pick)) {
            const hipError_t e = qai::tune_field(p->plans[i], p->tune[i], s, pick, nullptr);
            if (e != hipSuccess)
                return fail_hip(e, "autotune run");
            qai::cache_store(dims[i], pick);
        }
        best[key] = pick;
        p->tune[i] = pick;
    }
    if (each) {
        // every field: the pass-algorithm variants of its shape's setting
        for (int i = 0; i < p->n; ++i) {
            qai::Tuning pick;
            const hipError_t e = qai::refine_field(p->plans[i], p->tune[i], s, pick);
            if (e != hipSuccess)
                return fail_hip(e, "autotune run");
            p->tune[i] = pick;
        }
    }
    return QAI_OK;
}

int capture(qai_batch_plan* p)
{
    hipError_t e = hipStreamBeginCapture(p->capture, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess)
        return fail_hip(e, "hipStreamBeginCapture");
    hipError_t err = hipEventRecord(p->fork, p->capture);
    for (int k = 0; k < p->branches && err == hipSuccess; ++k)
        err = hipStreamWaitEvent(p->side[k], p->fork, 0);
    prof_suppress(true);
    for (size_t j = 0; j < p->order.size() && err == hipSuccess; ++j) {
        const int i = p->order[j];
        err = qai::run_plain(p->plans[i], p->tune[i], p->side[j % p->branches]);
    }
    prof_suppress(false);
    for (int k = 0; k < p->branches && err == hipSuccess; ++k) {
        err = hipEventRecord(p->join[k], p->side[k]);
        if (err == hipSuccess)
            err = hipStreamWaitEvent(p->capture, p->join[k], 0);
    }
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(p->capture, &g);
    if (err != hipSuccess) {
        if (g)
            (void)hipGraphDestroy(g);
        return fail_hip(err, "batch capture");
    }
    if (e != hipSuccess)
        return fail_hip(e, "hipStreamEndCapture");
    p->graph = g;
    e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess)
        return fail_hip(e, "hipGraphInstantiate");
    return QAI_OK;
}

} // namespace

extern "C" {

size_t qai_batch_workspace_bytes(int n, const int64_t (*dims)[3])
{
    if (n < 1 || !dims)
        return 0;
    size_t total = 0;
    for (int i = 0; i < n; ++i) {
        const size_t b = qai_workspace_bytes(dims[i]);
        if (b == 0)
            return 0;
        total += align256(b);
    }
    return total;
}

int qai_batch_plan_create(int n, const float* const* fields, const int64_t (*dims)[3], const float* ebs,
                          float* const* outs, const qai_params* params, uint32_t flags, void* ws, size_t ws_bytes,
                          void* stream, qai_batch_plan** plan)
{
    if (!plan)
        return fail(QAI_EINVAL, "plan is NULL");
    *plan = nullptr;
    if (n < 1 || !fields || !dims || !ebs || !outs)
        return fail(QAI_EINVAL, "a batch needs n >= 1 fields, dims, bounds and outputs");
    if (flags & ~(uint32_t)(QAI_BATCH_AUTOTUNE | QAI_BATCH_TUNE_EACH))
        return fail(QAI_EINVAL, "unknown batch flags 0x%x", flags);
    qai_params prm;
    int rc = check_params(params, &prm);
    if (rc)
        return rc;
    int64_t n_i;
    for (int i = 0; i < n; ++i) {
        if ((rc = check_dims(dims[i], &n_i)))
            return rc;
        if ((rc = check_eb(ebs[i])))
            return rc;
        if (!fields[i] || !outs[i])
            return fail(QAI_EINVAL, "field %d: null field or output", i);
        const float *f = fields[i], *o = outs[i];
        if (o < f + n_i && f < o + n_i)
            return fail(QAI_EINVAL, "field %d: a batch output may not overlap its input", i);
    }
    const size_t need = qai_batch_workspace_bytes(n, dims);
    if (!ws || ws_bytes < need)
        return fail(QAI_ENOWS, "batch workspace of %zu bytes needed, %zu given", need, ws ? ws_bytes : (size_t)0);
    if (((uintptr_t)ws & 255u) != 0)
        return fail(QAI_ENOWS, "workspace must be 256-byte aligned");

    qai_batch_plan* p = new qai_batch_plan();
    p->n = n;
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        release(p);
        return fail(QAI_ENODEV, "no usable GPU: %s", hipGetErrorString(e));
    }
    unsigned char* cur = (unsigned char*)ws;
    p->plans.resize(n);
    p->tune.resize(n);
    for (int i = 0; i < n; ++i)
        p->tune[i] = tuning_for(dims[i]);
    for (int i = 0; i < n; ++i) {
        qai::Plan1& pl = p->plans[i];
        pl = qai::Plan1{};
        pl.xq = fields[i];
        pl.out = outs[i];
        pl.nz = dims[i][0];
        pl.ny = dims[i][1];
        pl.nx = dims[i][2];
        pl.eb = ebs[i];
        pl.eta = prm.eta;
        pl.power = prm.power;
        ws_buffers(cur, pl);
        cur += align256(qai_workspace_bytes(dims[i]));
        p->order.push_back(i);
    }
    std::stable_sort(p->order.begin(), p->order.end(),
                     [&](int a, int b) { return voxels(dims[a]) > voxels(dims[b]); });
    p->branches = std::min(n, kMaxBranches);

    e = hipStreamCreateWithFlags(&p->capture, hipStreamNonBlocking);
    for (int k = 0; k < p->branches && e == hipSuccess; ++k) {
        hipStream_t s = nullptr;
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e == hipSuccess)
            p->side.push_back(s);
        hipEvent_t ev = nullptr;
        if (e == hipSuccess && (e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) == hipSuccess)
            p->join.push_back(ev);
    }
    if (e == hipSuccess)
        e = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming);
    if (e != hipSuccess) {
        release(p);
        return fail_hip(e, "batch streams");
    }
    if (flags & (QAI_BATCH_AUTOTUNE | QAI_BATCH_TUNE_EACH)) {
        prof_suppress(true);
        rc = autotune(p, dims, (hipStream_t)stream, (flags & QAI_BATCH_TUNE_EACH) != 0);
        prof_suppress(false);
        if (rc) {
            release(p);
            return rc;
        }
    }
    // the caller's stream must be idle before the capture stream records
    if ((e = hipStreamSynchronize((hipStream_t)stream)) != hipSuccess) {
        release(p);
        return fail_hip(e, "hipStreamSynchronize");
    }
    if ((rc = capture(p))) {
        release(p);
        return rc;
    }
    *plan = p;
    return QAI_OK;
}

int qai_batch_plan_launch(qai_batch_plan* plan, void* stream)
{
    if (!plan || !plan->exec)
        return fail(QAI_ESTATE, "no batch plan");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != plan->device)
        return fail(QAI_ESTATE, "the plan belongs to device %d", plan->device);
    hipError_t e = hipGraphLaunch(plan->exec, (hipStream_t)stream);
    if (e != hipSuccess)
        return fail_hip(e, "hipGraphLaunch");
    return QAI_OK;
}

int qai_batch_plan_launch_per_field(qai_batch_plan* plan, void* stream)
{
    if (!plan)
        return fail(QAI_ESTATE, "no batch plan");
    for (int i = 0; i < plan->n; ++i) {
        hipError_t e = qai::run_plain(plan->plans[i], plan->tune[i], (hipStream_t)stream);
        if (e != hipSuccess)
            return fail_hip(e, "kernel launch");
    }
    return QAI_OK;
}

int qai_batch_plan_tuning(const qai_batch_plan* plan, int field, qai_tuning* t)
{
    if (!plan || !t)
        return fail(QAI_EINVAL, "plan and t must not be NULL");
    if (field < 0 || field >= plan->n)
        return fail(QAI_EINVAL, "field %d outside [0, %d)", field, plan->n);
    return qai::api::tuning_to_abi(plan->tune[field], t);
}

void qai_batch_plan_destroy(qai_batch_plan* plan) { release(plan); }

} // extern "C"
