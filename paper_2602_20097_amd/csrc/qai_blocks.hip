// qai_blocks.hip -- the paper's block-decomposed strategies (Section VI-B)
// on one GPU: the field is cut into a grid of blocks, each processed as a
// field of its own, as the ranks of a distributed run would.
//
//  * embarrassingly parallel: every block runs the whole post-pass on its own
//    voxels (its faces are domain edges);
//  * approximate: every block works on its ghosted region (the block plus one
//    layer on each face that has a neighbour).  Step A reads the neighbours'
//    values in that layer (the first stencil exchange); after steps A and B
//    every block publishes the first EDT's words of its own voxels to a shared
//    word array, and each block copies its ghost layer back from it (the
//    second exchange: the neighbours' propagated signs) before steps C, D and
//    E.  Both EDTs stay local: ghost voxels lie on the region's edge, so they
//    are never sites.
// The exact strategy is the whole-field pass (qai_mitigate_ex).
// The blocks are independent between the exchanges, so their pipelines run
// concurrently on four side streams (one per hardware queue of the process),
// forked from and joined back to the caller's stream.
#include <map>
#include <mutex>
#include <vector>

#include "qai.h"
#include "qai_device.h"
#include "qai_kernels.h"

using namespace qai::api;

namespace qai {
namespace {

struct Box {
    int64_t o[3], e[3]; // origin and extent per axis (z, y, x)
};

// Side streams and fork/join events per device, created on first use and kept
// for the process (default priority).  A call holds the mutex while it
// enqueues, so concurrent calls never interleave their records and waits on
// the shared events.
constexpr int kSides = 4;
struct Sides {
    hipStream_t side[kSides] = {};
    hipEvent_t fork = nullptr, join[kSides] = {};
    Aux* aux[kSides] = {};    // per side stream: the side stream of its blocks' step E
};
std::mutex g_sides_mu;
std::map<int, Sides> g_sides;

hipError_t sides_for(int dev, Sides*& out)
{
    auto it = g_sides.find(dev);
    if (it != g_sides.end()) {
        out = &it->second;
        return hipSuccess;
    }
    Sides sd;
    hipError_t e = hipEventCreateWithFlags(&sd.fork, hipEventDisableTiming);
    for (int k = 0; k < kSides && e == hipSuccess; ++k) {
        e = hipStreamCreateWithFlags(&sd.side[k], hipStreamNonBlocking);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&sd.join[k], hipEventDisableTiming);
        if (e == hipSuccess) {
            Aux* x = new Aux();
            sd.aux[k] = x;
            e = hipStreamCreateWithFlags(&x->s, hipStreamNonBlocking);
            if (e == hipSuccess)
                e = hipEventCreateWithFlags(&x->fork, hipEventDisableTiming);
            if (e == hipSuccess)
                e = hipEventCreateWithFlags(&x->join, hipEventDisableTiming);
        }
    }
    if (e != hipSuccess)
        return e; // (what was created stays: a failed call is not retried here)
    out = &g_sides.emplace(dev, sd).first->second;
    return hipSuccess;
}

// the side streams wait for the work enqueued on s so far
hipError_t fork_sides(const Sides& sd, hipStream_t s)
{
    hipError_t e = hipEventRecord(sd.fork, s);
    for (int k = 0; k < kSides && e == hipSuccess; ++k)
        e = hipStreamWaitEvent(sd.side[k], sd.fork, 0);
    return e;
}

// s waits for the work enqueued on the side streams
hipError_t join_sides(const Sides& sd, hipStream_t s)
{
    hipError_t e = hipSuccess;
    for (int k = 0; k < kSides && e == hipSuccess; ++k) {
        e = hipEventRecord(sd.join[k], sd.side[k]);
        if (e == hipSuccess)
            e = hipStreamWaitEvent(s, sd.join[k], 0);
    }
    return e;
}

void bounds(int64_t n, int k, int i, int64_t& o, int64_t& e)
{
    const int64_t base = n / k, extra = n % k;
    e = base + (i < extra ? 1 : 0);
    o = (int64_t)i * base + (i < extra ? i : extra);
}

// The real box of block (iz, iy, ix) and its region (ghost layers where a
// neighbour exists, when ghost is set).
void block_boxes(const int64_t d[3], const int32_t k[3], const int idx[3], bool ghost, Box& real, Box& region)
{
    for (int a = 0; a < 3; ++a) {
        bounds(d[a], k[a], idx[a], real.o[a], real.e[a]);
        const int64_t lo = (ghost && real.o[a] > 0) ? real.o[a] - 1 : real.o[a];
        const int64_t hi = (ghost && real.o[a] + real.e[a] < d[a]) ? real.o[a] + real.e[a] + 1 : real.o[a] + real.e[a];
        region.o[a] = lo;
        region.e[a] = hi - lo;
    }
}

// Copy the region box of a global array into a dense local array (grid: x
// blocks of 256, y, z); with ghost_only, voxels of the real box are skipped.
__global__ __launch_bounds__(256) void k_region_copy(const uint32_t* __restrict__ src, int64_t gny, int64_t gnx,
                                                     Box reg, Box real, uint32_t* __restrict__ dst, int ghost_only)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t y = blockIdx.y, z = blockIdx.z;
    if (x >= reg.e[2])
        return;
    const int64_t gz = reg.o[0] + z, gy = reg.o[1] + y, gx = reg.o[2] + x;
    if (ghost_only && gz >= real.o[0] && gz < real.o[0] + real.e[0] && gy >= real.o[1] &&
        gy < real.o[1] + real.e[1] && gx >= real.o[2] && gx < real.o[2] + real.e[2])
        return;
    dst[(z * reg.e[1] + y) * reg.e[2] + x] = src[(gz * gny + gy) * gnx + gx];
}

// Store the real box of a dense local region array into the global array.
__global__ __launch_bounds__(256) void k_region_store(const uint32_t* __restrict__ src, Box reg, Box real,
                                                      uint32_t* __restrict__ dst, int64_t gny, int64_t gnx)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t y = blockIdx.y, z = blockIdx.z;
    if (x >= real.e[2])
        return;
    const int64_t gz = real.o[0] + z, gy = real.o[1] + y, gx = real.o[2] + x;
    const int64_t lz = gz - reg.o[0], ly = gy - reg.o[1], lx = gx - reg.o[2];
    dst[(gz * gny + gy) * gnx + gx] = src[(lz * reg.e[1] + ly) * reg.e[2] + lx];
}

hipError_t copy_region(const void* src, const int64_t d[3], const Box& reg, const Box& real, void* dst, bool ghost_only,
                       hipStream_t s)
{
    const dim3 grid((uint32_t)((reg.e[2] + 255) / 256), (uint32_t)reg.e[1], (uint32_t)reg.e[0]);
    return launch_checked(k_region_copy, grid, dim3(256), 0, s, (const uint32_t*)src, d[1], d[2], reg, real,
                          (uint32_t*)dst, ghost_only ? 1 : 0);
}

hipError_t store_region(const void* src, const Box& reg, const Box& real, void* dst, const int64_t d[3], hipStream_t s)
{
    const dim3 grid((uint32_t)((real.e[2] + 255) / 256), (uint32_t)real.e[1], (uint32_t)real.e[0]);
    return launch_checked(k_region_store, grid, dim3(256), 0, s, (const uint32_t*)src, reg, real, (uint32_t*)dst, d[1],
                          d[2]);
}

constexpr int kMaxBlocks = 4096;

// Workspace of one block: region copy of the field, region output, plain
// workspace; all 256-byte aligned.
size_t block_bytes(const Box& reg)
{
    const int64_t rd[3] = {reg.e[0], reg.e[1], reg.e[2]};
    const size_t n = (size_t)(reg.e[0] * reg.e[1] * reg.e[2]);
    return 2 * align256(4 * n) + align256(qai_workspace_bytes(rd));
}

int check_blocks(const int64_t dims[3], const int32_t blocks[3], int mode, int64_t* nb)
{
    int64_t n;
    int rc = check_dims(dims, &n);
    if (rc)
        return rc;
    if (!blocks)
        return fail(QAI_EINVAL, "blocks is NULL");
    if (mode != QAI_BLOCKS_EP && mode != QAI_BLOCKS_APPROX)
        return fail(QAI_EINVAL, "mode must be QAI_BLOCKS_EP or QAI_BLOCKS_APPROX");
    int64_t total = 1;
    for (int a = 0; a < 3; ++a) {
        if (blocks[a] < 1 || blocks[a] > dims[a])
            return fail(QAI_EINVAL, "blocks[%d] = %d outside [1, %lld]", a, blocks[a], (long long)dims[a]);
        total *= blocks[a];
    }
    if (total > kMaxBlocks)
        return fail(QAI_EINVAL, "at most %d blocks", kMaxBlocks);
    *nb = total;
    return QAI_OK;
}

} // namespace
} // namespace qai

extern "C" {

size_t qai_blocks_workspace_bytes(const int64_t dims[3], const int32_t blocks[3], int mode)
{
    int64_t nb;
    if (qai::check_blocks(dims, blocks, mode, &nb))
        return 0;
    size_t total = mode == QAI_BLOCKS_APPROX ? align256((size_t)(dims[0] * dims[1] * dims[2]) * 4) : 0;
    int idx[3];
    for (idx[0] = 0; idx[0] < blocks[0]; ++idx[0])
        for (idx[1] = 0; idx[1] < blocks[1]; ++idx[1])
            for (idx[2] = 0; idx[2] < blocks[2]; ++idx[2]) {
                qai::Box real, reg;
                qai::block_boxes(dims, blocks, idx, mode == QAI_BLOCKS_APPROX, real, reg);
                total += qai::block_bytes(reg);
            }
    return total;
}

int qai_mitigate_blocks(const float* field, const int64_t dims[3], float eb, const qai_params* params,
                        const int32_t blocks[3], int mode, void* ws, size_t ws_bytes, float* out, void* stream)
{
    clear_error();
    int64_t nb;
    int rc = qai::check_blocks(dims, blocks, mode, &nb);
    if (rc)
        return rc;
    const int64_t n = dims[0] * dims[1] * dims[2];
    if (!field || !out)
        return fail(QAI_EINVAL, "field and out must be device pointers");
    if ((rc = check_eb(eb)))
        return rc;
    qai_params prm;
    if ((rc = check_params(params, &prm)))
        return rc;
    const size_t need = qai_blocks_workspace_bytes(dims, blocks, mode);
    if (!ws || ws_bytes < need)
        return fail(QAI_ENOWS, "workspace of %zu bytes needed, %zu given", need, ws ? ws_bytes : (size_t)0);
    if (((uintptr_t)ws & 255u) != 0)
        return fail(QAI_ENOWS, "workspace must be 256-byte aligned");
    if (out != field && out < field + n && field < out + n)
        return fail(QAI_EINVAL, "out partly overlaps field");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fail(QAI_ENODEV, "no usable GPU: %s", hipGetErrorString(e));
    const hipStream_t s = (hipStream_t)stream;
    const bool approx = mode == QAI_BLOCKS_APPROX;

    struct Blk {
        qai::Box real, reg;
        qai::Plan1 plan;
        qai::Tuning tune;
        int w1;
    };
    std::vector<Blk> bl;
    bl.reserve((size_t)nb);
    unsigned char* cur = (unsigned char*)ws;
    uint32_t* shared_words = nullptr;
    if (approx) {
        shared_words = (uint32_t*)cur;
        cur += align256((size_t)n * 4);
    }
    int idx[3];
    for (idx[0] = 0; idx[0] < blocks[0]; ++idx[0])
        for (idx[1] = 0; idx[1] < blocks[1]; ++idx[1])
            for (idx[2] = 0; idx[2] < blocks[2]; ++idx[2]) {
                Blk b;
                qai::block_boxes(dims, blocks, idx, approx, b.real, b.reg);
                const size_t rn = (size_t)(b.reg.e[0] * b.reg.e[1] * b.reg.e[2]);
                b.plan = qai::Plan1{};
                b.plan.xq = (const float*)cur;
                b.plan.out = (float*)(cur + align256(4 * rn));
                b.plan.nz = b.reg.e[0];
                b.plan.ny = b.reg.e[1];
                b.plan.nx = b.reg.e[2];
                b.plan.eb = eb;
                b.plan.eta = prm.eta;
                b.plan.power = prm.power;
                ws_buffers(cur + 2 * align256(4 * rn), b.plan);
                const int64_t rd[3] = {b.reg.e[0], b.reg.e[1], b.reg.e[2]};
                b.tune = tuning_for(rd);
                b.w1 = 0;
                cur += qai::block_bytes(b.reg);
                bl.push_back(b);
            }

#define QAI_BTRY(expr)                                   \
    do {                                                 \
        if ((e = (expr)) != hipSuccess)                  \
            return fail_hip(e, "block pipeline launch"); \
    } while (0)
    std::lock_guard<std::mutex> lk(qai::g_sides_mu);
    qai::Sides* sd = nullptr;
    QAI_BTRY(qai::sides_for(dev, sd));
    for (Blk& b : bl)
        QAI_BTRY(qai::copy_region(field, dims, b.reg, b.real, (void*)b.plan.xq, false, s));
    if (!qai::stream_capturing(s))
        for (size_t i = 0; i < bl.size(); ++i)
            bl[i].plan.aux = sd->aux[i % qai::kSides]; // guarded by g_sides_mu
    QAI_BTRY(qai::fork_sides(*sd, s));
    if (!approx) {
        for (size_t i = 0; i < bl.size(); ++i)
            QAI_BTRY(qai::run_plain(bl[i].plan, bl[i].tune, sd->side[i % qai::kSides]));
        QAI_BTRY(qai::join_sides(*sd, s));
    } else {
        for (size_t i = 0; i < bl.size(); ++i)
            QAI_BTRY(qai::run_part1(bl[i].plan, bl[i].tune, sd->side[i % qai::kSides], &bl[i].w1));
        QAI_BTRY(qai::join_sides(*sd, s));
        // exchange: every block's own first-EDT words to the shared array ...
        for (Blk& b : bl) {
            uint32_t* bufs[3] = {b.plan.bufA, b.plan.bufB, b.plan.bufC};
            QAI_BTRY(qai::store_region(bufs[b.w1], b.reg, b.real, shared_words, dims, s));
        }
        // ... and its ghost layer back from the neighbours' words
        for (Blk& b : bl) {
            uint32_t* bufs[3] = {b.plan.bufA, b.plan.bufB, b.plan.bufC};
            QAI_BTRY(qai::copy_region(shared_words, dims, b.reg, b.real, bufs[b.w1], true, s));
        }
        QAI_BTRY(qai::fork_sides(*sd, s));
        for (size_t i = 0; i < bl.size(); ++i)
            QAI_BTRY(qai::run_part2(bl[i].plan, bl[i].tune, sd->side[i % qai::kSides], bl[i].w1));
        QAI_BTRY(qai::join_sides(*sd, s));
    }
    for (Blk& b : bl)
        QAI_BTRY(qai::store_region(b.plan.out, b.reg, b.real, out, dims, s));
#undef QAI_BTRY
    return QAI_OK;
}

} // extern "C"
