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
// The sums run in FP64 over a fixed grid and a fixed reduction tree, so the
// result does not depend on scheduling.
#include <math.h>

#include "qai.h"
#include "qai_device.h"
#include "qai_kernels.h"

namespace qai {

constexpr int kGradBlocks = 1024;
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

__global__ __launch_bounds__(kGradThreads) void k_grad_partial(const float* __restrict__ g,
                                                                const uint32_t* __restrict__ w1,
                                                                const uint32_t* __restrict__ w2, int64_t n,
                                                                float eb, float eta, float power,
                                                                double* __restrict__ partial)
{
    __shared__ double sh[kGradThreads];
    double se = 0.0, sp = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t a = w1[i];
        const int s = word_sign(a);
        if (s == 0)
            continue;
        const uint32_t b = w2[i];
        const bool none2 = (b == QAI_WORD_INF);
        const uint32_t d1 = word_d2(a), d2 = none2 ? 0u : word_d2(b);
        const float wt = idw_weight(d1, false, d2, none2, power);
        const double gs = (double)g[i] * (double)s;
        se += gs * (double)wt * (double)eb;
        if (d1 != 0u && !none2 && d2 != 0u) {
            const double lr = 0.5 * (log((double)d1) - log((double)d2)); // ln(k1 / k2)
            sp += gs * (double)eta * (double)eb * (-(double)wt * (1.0 - (double)wt) * lr);
        }
    }
    se = block_sum(se, sh);
    sp = block_sum(sp, sh);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = se;
        partial[2 * blockIdx.x + 1] = sp;
    }
}

__global__ __launch_bounds__(kGradThreads) void k_grad_final(const double* __restrict__ partial,
                                                              float* __restrict__ out)
{
    __shared__ double sh[kGradThreads];
    double se = 0.0, sp = 0.0;
    for (int b = threadIdx.x; b < kGradBlocks; b += kGradThreads) {
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
    const hipError_t e = launch_checked(k_grad_partial, dim3(kGradBlocks), dim3(kGradThreads), 0, s, g, w1, w2, n, eb,
                                        eta, power, partial);
    if (e != hipSuccess)
        return e;
    return launch_checked(k_grad_final, dim3(1), dim3(kGradThreads), 0, s, (const double*)partial, out);
}

} // namespace qai
