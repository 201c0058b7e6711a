// qai_quality.hip -- the quality metrics of the paper's evaluation on the
// GPU: SSIM (Eq. 3: per-window means, sample variances and covariance of the
// range-normalised fields, c1 = 1e-4, c2 = 9e-4, windows of 7 voxels per axis
// moved by 2, averaged over all windows) and PSNR (Eq. 4), for comparing an
// original field with a decompressed or compensated one.
//
// Readings: both fields are normalised by the original's range
// ((x - min) / (max - min)); sample moments divide by m - 1 for m voxels per
// window; an axis shorter than 7 takes its whole extent as the window.
//
// Two passes over the fields: the first reduces min and max of the original
// and the squared differences (PSNR, MSE); the second marches z-planes
// through tiles of 16 x 16 window positions: a plane's row sums over the
// x-window (FP64, from the plane tile staged in LDS), then the y-window sums
// per position, added to the (at most four) windows along z the plane belongs
// to; each window that completes on a plane adds its SSIM.  All sums are FP64 and the
// reduction order is fixed by the shape, so results are deterministic.
#include <math.h>

#include "qai.h"
#include "qai_device.h"
#include "qai_kernels.h"

using namespace qai::api;

namespace qai {
namespace {

constexpr int kQW = 7, kQS = 2;       // window and stride
constexpr int kRedBlocks = 2048, kRedThreads = 256;
constexpr int kTile = 16;             // window positions per tile side
constexpr int kZChunk = 32;           // window positions along z per block
constexpr size_t kRangeOffset = 0;    // first pass: 3 doubles per block
constexpr size_t kResultOffset = 3 * kRedBlocks * sizeof(double);  // min, max, sse (3 doubles)
constexpr size_t kSsimOffset = 64 * 1024;                          // second pass: 1 double per block

struct QGeom {
    int64_t nz, ny, nx;
    int wz, wy, wx;        // window extents
    int64_t pz, py, px;    // window positions per axis
    int64_t tiles_y, tiles_x, chunks_z;
};

QGeom geom(const int64_t d[3])
{
    QGeom g;
    g.nz = d[0];
    g.ny = d[1];
    g.nx = d[2];
    g.wz = (int)(g.nz < kQW ? g.nz : kQW);
    g.wy = (int)(g.ny < kQW ? g.ny : kQW);
    g.wx = (int)(g.nx < kQW ? g.nx : kQW);
    g.pz = (g.nz - g.wz) / kQS + 1;
    g.py = (g.ny - g.wy) / kQS + 1;
    g.px = (g.nx - g.wx) / kQS + 1;
    g.tiles_y = (g.py + kTile - 1) / kTile;
    g.tiles_x = (g.px + kTile - 1) / kTile;
    g.chunks_z = (g.pz + kZChunk - 1) / kZChunk;
    return g;
}

__device__ __forceinline__ double block_sum(double v, double* sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (t < s)
            sh[t] += sh[t + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ float block_min(float v, float* sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (t < s)
            sh[t] = fminf(sh[t], sh[t + s]);
        __syncthreads();
    }
    const float r = sh[0];
    __syncthreads();
    return r;
}

// First pass: min and max of the original, sum of squared differences.
template <bool VEC>
__global__ __launch_bounds__(kRedThreads) void k_range_sse(const float* __restrict__ a, const float* __restrict__ b,
                                                           int64_t n, double* __restrict__ part)
{
    __shared__ double shd[kRedThreads];
    __shared__ float shf[kRedThreads];
    float lo = INFINITY, hi = -INFINITY;
    double sse = 0.0;
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    int64_t tail = 0;
    if (VEC) {
        const float4* a4 = reinterpret_cast<const float4*>(a);
        const float4* b4 = reinterpret_cast<const float4*>(b);
        const int64_t n4 = n >> 2;
        for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n4; q += step) {
            const float4 u = a4[q], v = b4[q];
            lo = fminf(lo, fminf(fminf(u.x, u.y), fminf(u.z, u.w)));
            hi = fmaxf(hi, fmaxf(fmaxf(u.x, u.y), fmaxf(u.z, u.w)));
            const double dx = (double)u.x - (double)v.x, dy = (double)u.y - (double)v.y;
            const double dz = (double)u.z - (double)v.z, dw = (double)u.w - (double)v.w;
            sse += (dx * dx + dy * dy) + (dz * dz + dw * dw);
        }
        tail = n4 << 2;
    }
    for (int64_t i = tail + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) {
        const float u = a[i];
        lo = fminf(lo, u);
        hi = fmaxf(hi, u);
        const double d = (double)u - (double)b[i];
        sse += d * d;
    }
    sse = block_sum(sse, shd);
    lo = block_min(lo, shf);
    hi = -block_min(-hi, shf);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = (double)lo;
        part[3 * blockIdx.x + 1] = (double)hi;
        part[3 * blockIdx.x + 2] = sse;
    }
}

__global__ __launch_bounds__(kRedThreads) void k_range_final(const double* __restrict__ part, int nb,
                                                             double* __restrict__ res)
{
    __shared__ double sh[kRedThreads];
    __shared__ float shf[kRedThreads];
    float lo = INFINITY, hi = -INFINITY;
    double sse = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        lo = fminf(lo, (float)part[3 * b]);
        hi = fmaxf(hi, (float)part[3 * b + 1]);
        sse += part[3 * b + 2];
    }
    sse = block_sum(sse, sh);
    lo = block_min(lo, shf);
    hi = -block_min(-hi, shf);
    if (threadIdx.x == 0) {
        res[0] = (double)lo;
        res[1] = (double)hi;
        res[2] = sse;
    }
}

// Second pass.  Block (tx, ty, cz): window positions wy in [ty*16, +16),
// wx in [tx*16, +16), wz in [cz*32, +32); thread (ly, lx) owns one (wy, wx).
// Planes are taken in groups of eight aligned to z = 0 mod 8: a plane
// belongs to the windows starting at most 6 planes before it, at most four
// of them, each held in accumulator slot (start / 2) mod 4 -- a static index
// within the group.  The next plane's tile is loaded into registers while the
// current one is summed (two LDS tile buffers, two barriers per plane).
constexpr int kRows = (kTile - 1) * kQS + kQW; // 37 staged rows / columns per plane
constexpr int kStage = (kRows * kRows + 255) / 256; // tile elements per thread and field

__global__ __launch_bounds__(256) void k_ssim(const float* __restrict__ a, const float* __restrict__ b, QGeom g,
                                              const double* __restrict__ rng, double* __restrict__ part)
{
    __shared__ float ta[2][kRows * kRows], tb[2][kRows * kRows];
    __shared__ double xs[5][kRows][kTile];
    __shared__ double sh[256];
    const int t = threadIdx.x;
    const int lx = t & (kTile - 1), ly = t >> 4;
    const int64_t bx = blockIdx.x, by = blockIdx.y, cz = blockIdx.z;
    const int64_t wx = bx * kTile + lx, wy = by * kTile + ly;
    const bool mine = wx < g.px && wy < g.py;
    const int64_t x0 = bx * kTile * kQS, y0 = by * kTile * kQS;
    const int cols = (int)min((int64_t)kRows, g.nx - x0), rows = (int)min((int64_t)kRows, g.ny - y0);
    const int64_t wz0 = cz * kZChunk, wz1 = min(g.pz, wz0 + kZChunk);
    const int64_t z0 = wz0 * kQS, z1 = (wz1 - 1) * kQS + g.wz; // planes this block reads; z0 = 0 mod 8
    const double lo = rng[0];
    const double inv = 1.0 / (rng[1] - rng[0]);
    const int m = g.wz * g.wy * g.wx;
    const double rm = 1.0 / (double)m, rm1 = 1.0 / (double)(m - 1);
    const int wz = g.wz;
    double acc[4][5];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int q = 0; q < 5; ++q)
            acc[k][q] = 0.0;
    double total = 0.0;

    // this thread's share of a plane tile: elements t, t + 256, ... of rows x cols
    float ra[kStage], rb[kStage];
    auto fetch = [&](int64_t z) {
        const int64_t pb = (min(z, g.nz - 1) * g.ny + y0) * g.nx + x0;
#pragma unroll
        for (int e = 0; e < kStage; ++e) {
            const int i = t + e * 256;
            const int r = i / cols, c = i - r * cols;
            const bool in = i < rows * cols;
            const int64_t gi = pb + (in ? (int64_t)r * g.nx + c : 0);
            ra[e] = a[gi];
            rb[e] = b[gi];
        }
    };
    auto stage = [&](int buf) {
#pragma unroll
        for (int e = 0; e < kStage; ++e) {
            const int i = t + e * 256;
            if (i < rows * cols) {
                const int r = i / cols, c = i - r * cols;
                ta[buf][r * kRows + c] = ra[e];
                tb[buf][r * kRows + c] = rb[e];
            }
        }
    };

    fetch(z0);
    int buf = 0;
    for (int64_t zb = z0; zb < z1; zb += 8) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int64_t z = zb + k;
            if (z >= z1)
                break;
            stage(buf);
            __syncthreads();
            if (z + 1 < z1)
                fetch(z + 1);
            // row sums over the x-window at every window column of the tile
            for (int i = t; i < rows * kTile; i += 256) {
                const int r = i >> 4, cc = i & (kTile - 1), c = cc * kQS;
                double su = 0.0, sv = 0.0, suu = 0.0, svv = 0.0, suv = 0.0;
                if (c + g.wx <= cols) {
                    for (int j = 0; j < g.wx; ++j) {
                        const double u = ((double)ta[buf][r * kRows + c + j] - lo) * inv;
                        const double v = ((double)tb[buf][r * kRows + c + j] - lo) * inv;
                        su += u;
                        sv += v;
                        suu += u * u;
                        svv += v * v;
                        suv += u * v;
                    }
                }
                xs[0][r][cc] = su;
                xs[1][r][cc] = sv;
                xs[2][r][cc] = suu;
                xs[3][r][cc] = svv;
                xs[4][r][cc] = suv;
            }
            __syncthreads();
            double pl[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
            if (mine) {
                for (int j = 0; j < g.wy; ++j)
#pragma unroll
                    for (int q = 0; q < 5; ++q)
                        pl[q] += xs[q][ly * kQS + j][lx];
            }
            // the windows starting d = 0..6 planes before z (even starts only)
#pragma unroll
            for (int d = 0; d < kQW; ++d) {
                if (((k - d) & 1) != 0)
                    continue;                           // odd start: not a window
                const int slot = ((k - d + 8) >> 1) & 3; // static: zb = 0 mod 8
                const int64_t st = z - d;
                if (d >= wz || st < z0 || st < 0 || st / kQS >= wz1)
                    continue;                           // uniform over the block
#pragma unroll
                for (int q = 0; q < 5; ++q)
                    acc[slot][q] = (d == 0 ? 0.0 : acc[slot][q]) + pl[q];
                if (d == wz - 1 && mine) {
                    const double* w = acc[slot];
                    const double mu = w[0] * rm, mv = w[1] * rm;
                    const double vu = (w[2] - w[0] * mu) * rm1, vv = (w[3] - w[1] * mv) * rm1;
                    const double cv = (w[4] - w[0] * mv) * rm1;
                    total += ((2.0 * mu * mv + 1e-4) * (2.0 * cv + 9e-4)) /
                             ((mu * mu + mv * mv + 1e-4) * (vu + vv + 9e-4));
                }
            }
            buf ^= 1;
        }
    }
    total = block_sum(total, sh);
    if (t == 0)
        part[(cz * g.tiles_y + by) * g.tiles_x + bx] = total;
}

__global__ __launch_bounds__(256) void k_ssim_final(const double* __restrict__ part, int64_t nb, double windows,
                                                    const double* __restrict__ rs, double n, double* __restrict__ out)
{
    __shared__ double sh[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < nb; i += blockDim.x)
        s += part[i];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) {
        const double range = rs[1] - rs[0];
        const double mse = rs[2] / n;
        out[0] = range > 0.0 ? s / windows : NAN;
        out[1] = mse > 0.0 ? 20.0 * log10(range / sqrt(mse)) : INFINITY;
        out[2] = mse;
        out[3] = range;
    }
}

} // namespace
} // namespace qai

extern "C" {

size_t qai_quality_workspace_bytes(const int64_t dims[3])
{
    int64_t n;
    if (!dims || check_dims(dims, &n))
        return 0;
    const qai::QGeom g = qai::geom(dims);
    return qai::kSsimOffset + align256((size_t)(g.tiles_x * g.tiles_y * g.chunks_z) * sizeof(double));
}

int qai_quality(const float* orig, const float* dec, const int64_t dims[3], void* ws, size_t ws_bytes,
                double* result, void* stream)
{
    clear_error();
    int64_t n;
    int rc = check_dims(dims, &n);
    if (rc)
        return rc;
    if (!orig || !dec || !result)
        return fail(QAI_EINVAL, "orig, dec and result must be device pointers");
    const qai::QGeom g = qai::geom(dims);
    if ((int64_t)g.wz * g.wy * g.wx < 2)
        return fail(QAI_EDIMS, "a window needs at least two voxels");
    if (g.tiles_y > 65535 || g.chunks_z > 65535)
        return fail(QAI_EDIMS, "field too large for the SSIM grid");
    const size_t need = qai_quality_workspace_bytes(dims);
    if (!ws || ws_bytes < need)
        return fail(QAI_ENOWS, "workspace of %zu bytes needed, %zu given", need, ws ? ws_bytes : (size_t)0);
    if (((uintptr_t)ws & 255u) != 0)
        return fail(QAI_ENOWS, "workspace must be 256-byte aligned");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fail(QAI_ENODEV, "no usable GPU: %s", hipGetErrorString(e));
    const hipStream_t s = (hipStream_t)stream;
    unsigned char* w = (unsigned char*)ws;
    double* part = (double*)(w + qai::kRangeOffset);
    double* res = (double*)(w + qai::kResultOffset);
    double* sp = (double*)(w + qai::kSsimOffset);
    const bool vec = (((uintptr_t)orig | (uintptr_t)dec) & 15u) == 0;
    int64_t nb = ((vec ? (n + 3) / 4 : n) + qai::kRedThreads - 1) / qai::kRedThreads;
    nb = nb < 1 ? 1 : (nb > qai::kRedBlocks ? qai::kRedBlocks : nb);
    e = vec ? qai::launch_checked(qai::k_range_sse<true>, dim3((uint32_t)nb), dim3(qai::kRedThreads), 0, s, orig, dec,
                                  n, part)
            : qai::launch_checked(qai::k_range_sse<false>, dim3((uint32_t)nb), dim3(qai::kRedThreads), 0, s, orig,
                                  dec, n, part);
    if (e == hipSuccess)
        e = qai::launch_checked(qai::k_range_final, dim3(1), dim3(qai::kRedThreads), 0, s, (const double*)part,
                                (int)nb, res);
    if (e == hipSuccess)
        e = qai::launch_checked(qai::k_ssim, dim3((uint32_t)g.tiles_x, (uint32_t)g.tiles_y, (uint32_t)g.chunks_z),
                                dim3(256), 0, s, orig, dec, g, (const double*)res, sp);
    const int64_t nbs = g.tiles_x * g.tiles_y * g.chunks_z;
    if (e == hipSuccess)
        e = qai::launch_checked(qai::k_ssim_final, dim3(1), dim3(256), 0, s, (const double*)sp, nbs,
                                (double)(g.px * g.py * g.pz), (const double*)res, (double)n, result);
    return e == hipSuccess ? QAI_OK : fail_hip(e, "quality launch");
}

} // extern "C"
