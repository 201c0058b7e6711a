// qai_grad.hip -- adjoint of step E (a project addition; the paper tunes eta
// by an offline sweep, Section V-E).
//
// out_i = x'_i + w_i S_i eta eb with w_i = k1^-p / (k1^-p + k2^-p).  The EDT
// distances k1, k2 and the signs S are piecewise constant in the data and are
// held fixed, so
//   dout_i/dx'_i = 1,
//   dL/deta  = sum_i g_i w_i S_i eb,
//   dL/dp    = sum_i g_i S_i eta eb dw_i/dp,  dw/dp = -w (1 - w) ln(k1/k2),
// with dw/dp = 0 wherever w is pinned (on B1, on B2, or with no B2).
// The sums run in FP64 over a grid fixed by n and a fixed reduction tree, so
// the result does not depend on scheduling.
#include <math.h>

#include "qai.h"
#include "qai_device.h"
#include "qai_kernels.h"

namespace qai {

constexpr int kGradBlocks = 2048; // partial sums: 2 doubles each, 32 KiB of the workspace header
constexpr int kGradThreads = 256;

__device__ __forceinline__ double block_sum(double v, double* sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = kGradThreads / 2; s > 0; s >>= 1) {
        if (t < s)
            sh[t] += sh[t + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// One voxel's terms: g S w eb (into se) and g S eta eb dw/dp (into sp).  The
// log ratio ln(k1/k2) = ln(d1^2/d2^2) / 2 is taken in FP32 on the rounded
// ratio (relative error of the term about 1e-7); the sums are FP64.
__device__ __forceinline__ void grad_terms(float g, uint32_t a, uint32_t b, float eb, float eta, float power,
                                           double& se, double& sp)
{
    const int s = word_sign(a);
    if (s == 0)
        return;
    const bool none2 = (b == QAI_WORD_INF);
    const uint32_t d1 = word_d2(a), d2 = none2 ? 0u : word_d2(b);
    const float wt = idw_weight(d1, false, d2, none2, power);
    const double gs = (double)g * (double)s;
    se += gs * (double)wt * (double)eb;
    if (d1 != 0u && !none2 && d2 != 0u) {
        const float lr = 0.5f * logf((float)d1 / (float)d2);
        sp += gs * (double)eta * (double)eb * (-(double)wt * (1.0 - (double)wt) * (double)lr);
    }
}

// Four voxels per thread and step with 16-byte loads of g and w1; the w2
// words of a quad are fetched only when one of its voxels has S != 0 (the
// only voxels whose terms are not zero).  VEC = false: one voxel per step
// (fields or gradients not 16-byte aligned).
template <bool VEC>
__global__ __launch_bounds__(kGradThreads) void k_grad_partial(const float* __restrict__ g,
                                                                const uint32_t* __restrict__ w1,
                                                                const uint32_t* __restrict__ w2, int64_t n,
                                                                float eb, float eta, float power,
                                                                double* __restrict__ partial)
{
    __shared__ double sh[kGradThreads];
    double se = 0.0, sp = 0.0;
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    int64_t tail = 0;
    if (VEC) {
        const int64_t n4 = n >> 2;
        const float4* g4 = reinterpret_cast<const float4*>(g);
        const uint4* a4 = reinterpret_cast<const uint4*>(w1);
        const uint4* b4 = reinterpret_cast<const uint4*>(w2);
        for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n4; q += step) {
            const uint4 a = a4[q];
            const float4 gv = g4[q];
            const bool any = ((a.x != QAI_WORD_INF) && (a.x & 3u)) || ((a.y != QAI_WORD_INF) && (a.y & 3u)) ||
                             ((a.z != QAI_WORD_INF) && (a.z & 3u)) || ((a.w != QAI_WORD_INF) && (a.w & 3u));
            if (!any)
                continue;
            const uint4 b = b4[q];
            grad_terms(gv.x, a.x, b.x, eb, eta, power, se, sp);
            grad_terms(gv.y, a.y, b.y, eb, eta, power, se, sp);
            grad_terms(gv.z, a.z, b.z, eb, eta, power, se, sp);
            grad_terms(gv.w, a.w, b.w, eb, eta, power, se, sp);
        }
        tail = n4 << 2;
    }
    for (int64_t i = tail + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) {
        const uint32_t a = w1[i];
        if (word_sign(a) == 0)
            continue;
        grad_terms(g[i], a, w2[i], eb, eta, power, se, sp);
    }
    se = block_sum(se, sh);
    sp = block_sum(sp, sh);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = se;
        partial[2 * blockIdx.x + 1] = sp;
    }
}

__global__ __launch_bounds__(kGradThreads) void k_grad_final(const double* __restrict__ partial, int nblocks,
                                                              float* __restrict__ out)
{
    __shared__ double sh[kGradThreads];
    double se = 0.0, sp = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kGradThreads) {
        se += partial[2 * b];
        sp += partial[2 * b + 1];
    }
    se = block_sum(se, sh);
    sp = block_sum(sp, sh);
    if (threadIdx.x == 0) {
        out[0] = (float)se;
        out[1] = (float)sp;
    }
}

hipError_t launch_backward(const float* g, const uint32_t* w1, const uint32_t* w2, int64_t n, float eb, float eta,
                           float power, double* partial, float* out, hipStream_t s)
{
    const bool vec = (((uintptr_t)g | (uintptr_t)w1 | (uintptr_t)w2) & 15u) == 0;
    const int64_t units = vec ? (n + 3) / 4 : n;
    int64_t nb = (units + kGradThreads - 1) / kGradThreads;
    nb = nb < 1 ? 1 : (nb > kGradBlocks ? kGradBlocks : nb);
    const hipError_t e =
        vec ? launch_checked(k_grad_partial<true>, dim3((uint32_t)nb), dim3(kGradThreads), 0, s, g, w1, w2, n, eb, eta,
                             power, partial)
            : launch_checked(k_grad_partial<false>, dim3((uint32_t)nb), dim3(kGradThreads), 0, s, g, w1, w2, n, eb,
                             eta, power, partial);
    if (e != hipSuccess)
        return e;
    return launch_checked(k_grad_final, dim3(1), dim3(kGradThreads), 0, s, (const double*)partial, (int)nb, out);
}

} // namespace qai
