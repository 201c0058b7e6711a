// qai_plain.hip -- kernels of the plain QAI post-pass for gfx950.
//
// Stage map (Algorithm 4 of the paper):
//   k_seed_*<0>      step A (Algorithm 2) fused with the x pass of step B:
//                    x' -> q -> B1 and S_B by a 6-neighbour stencil, then
//                    each voxel's nearest B1 voxel on its x-line.
//   k_env_*          remaining passes of step B: exact 1-D minimisation of
//                    g(j) + (i - j)^2 along y, then z (Algorithm 1's result,
//                    sign payload carried along).
//   k_seed_*<1>      step C (Algorithm 3): propagated S read from the final
//                    words, B2 by a 6-neighbour stencil, then the x pass of
//                    step D.
//   k_env_*          the y pass of step D, then either the z pass and
//                    k_interp (step E), or, for a 3-D call without taps,
//                    k_interp_own (or k_interp_pre, alongside the y pass) /
//                    k_interp_far: step E with the z pass done only where
//                    the weight depends on it.
// No dense contraction exists on this path: the stencil and scan kernels are
// bound by VALU issue, the envelope and search kernels by dependent latency,
// the streaming ones by HBM.
#include "qai_code.h"
#include "qai_device.h"
#include "qai_kernels.h"
#include <algorithm>
#include <type_traits>

#define QAI_TRY(expr)                   \
    do {                                \
        hipError_t e_ = (expr);         \
        if (e_ != hipSuccess)           \
            return e_;                  \
    } while (0)

namespace qai {

// ------------------------------------------------------------------ seeds
// One wave per x-line.  The line is visited in groups of 8 chunks of 64
// voxels; all stencil loads of a group are issued together.  Forward over
// the chunks: stencil, site flags by ballot, per-chunk masks, site codes and
// the last site before each chunk kept in LDS.  Backward: the nearest site to
// the left (highest set bit at or below the lane, else the carried one) and
// to the right; the left one wins ties (lower x, as Algorithm 1's strict
// query comparison).  Lanes past the end of the line read a valid word and
// ignore it.
template <int MODE>
__device__ __forceinline__ int seed_key(const SeedArgs& a, int64_t i, bool& bad)
{
    if (MODE == 0)
        return recover_q(a.xq[i], a.inv2eb, a.two_eb, bad);
    return word_sign(a.w1[i]);
}

template <int MODE>
__global__ __launch_bounds__(256) void k_seed_xscan(SeedArgs a)
{
    constexpr int CG = 8; // chunks per load group
    extern __shared__ __align__(16) unsigned char smem[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t nx = a.nx, ny = a.ny, nz = a.nz;
    const int nch = (int)((nx + 63) >> 6);
    const size_t code_bytes = (MODE == 0) ? (size_t)nch * 64 : 0;
    const size_t per_wave = (code_bytes + (size_t)nch * 12 + 15) & ~(size_t)15;
    unsigned char* codes = smem + (size_t)wave * per_wave;
    uint64_t* masks = (uint64_t*)(codes + code_bytes);
    int* carry = (int*)(masks + nch);
    const int64_t lines = ny * nz;
    const int64_t plane = nx * ny;
    const bool hy = ny > 1, hz = nz > 1, hx = nx > 1;

    for (uint64_t t = blockIdx.x; t < a.ngroups; t += gridDim.x) {
        const uint64_t grp = xcd_remap(t, a.ngroups);
        const int64_t line = (int64_t)grp * a.waves + wave;
        if (line >= lines)
            continue;
        const int64_t y = line % ny, z = line / ny;
        const int64_t base = line * nx;
        const bool line_in = (!hy || (y >= 1 && y <= ny - 2)) && (!hz || (z >= 1 && z <= nz - 2));
        bool bad = false;

        int last = -1;    // last site before the current chunk
        int kprev = 0;    // key at x = 64c - 1
        for (int c0 = 0; c0 < nch; c0 += CG) {
            int kc[CG], ky0[CG], ky1[CG], kz0[CG], kz1[CG];
            uint32_t wc[CG];
#pragma unroll
            for (int k = 0; k < CG; ++k) {
                const int64_t x = (int64_t)(c0 + k) * 64 + lane;
                const int64_t xs = x < nx ? x : nx - 1;   // clamped: always a valid address
                if (MODE == 0) {
                    kc[k] = recover_q(a.xq[base + xs], a.inv2eb, a.two_eb, bad);
                    wc[k] = 0u;
                } else {
                    wc[k] = a.w1[base + xs];
                    kc[k] = word_sign(wc[k]);
                }
                if (line_in) {
                    ky0[k] = hy ? seed_key<MODE>(a, base + xs - nx, bad) : kc[k];
                    ky1[k] = hy ? seed_key<MODE>(a, base + xs + nx, bad) : kc[k];
                    kz0[k] = hz ? seed_key<MODE>(a, base + xs - plane, bad) : kc[k];
                    kz1[k] = hz ? seed_key<MODE>(a, base + xs + plane, bad) : kc[k];
                } else {
                    ky0[k] = ky1[k] = kz0[k] = kz1[k] = kc[k];
                }
            }
#pragma unroll
            for (int k = 0; k < CG; ++k) {
                const int c = c0 + k;
                if (c >= nch)
                    break;
                const int64_t x = (int64_t)c * 64 + lane;
                const bool valid = x < nx;
                int km = __shfl_up(kc[k], 1);
                int kp = __shfl_down(kc[k], 1);
                const int knext = (k + 1 < CG) ? __shfl(kc[k + 1 < CG ? k + 1 : k], 0) : 0;
                if (lane == 0)
                    km = kprev;
                if (lane == 63 && x + 1 < nx)
                    kp = (k + 1 < CG) ? knext : seed_key<MODE>(a, base + x + 1, bad);
                kprev = __shfl(kc[k], 63);

                const bool x_in = !hx || (x >= 1 && x <= nx - 2);
                bool site = false;
                int sgn = 0;
                if (valid && line_in && x_in) {
                    if (MODE == 0) {
                        // Algorithm 2: boundary if some 6-neighbour index differs; sign of the
                        // first differing neighbour (+x, -x, +y, -y, +z, -z); discarded where
                        // an absolute central difference reaches 1 (|q+ - q-| >= 2).
                        const int q = kc[k];
                        int first = 0;
                        if (hx)
                            first = (kp != q) ? kp - q : ((km != q) ? km - q : 0);
                        if (hy && first == 0)
                            first = (ky1[k] != q) ? ky1[k] - q : ((ky0[k] != q) ? ky0[k] - q : 0);
                        if (hz && first == 0)
                            first = (kz1[k] != q) ? kz1[k] - q : ((kz0[k] != q) ? kz0[k] - q : 0);
                        const bool steep = (hx && abs(kp - km) >= 2) || (hy && abs(ky1[k] - ky0[k]) >= 2) ||
                                           (hz && abs(kz1[k] - kz0[k]) >= 2);
                        if (first != 0) {
                            site = true;
                            sgn = steep ? 0 : (first > 0 ? 1 : -1);
                        }
                    } else {
                        // Algorithm 3's GetBoundary(S): interior voxels outside B1 whose
                        // propagated sign differs from a 6-neighbour's.
                        const int sc = kc[k];
                        const bool on_b1 = (wc[k] != QAI_WORD_INF) && (word_d2(wc[k]) == 0u);
                        site = !on_b1 && ((hx && (kp != sc || km != sc)) || (hy && (ky0[k] != sc || ky1[k] != sc)) ||
                                          (hz && (kz0[k] != sc || kz1[k] != sc)));
                    }
                }
                if (MODE == 0)
                    codes[c * 64 + lane] = (unsigned char)sign_code(sgn);
                const uint64_t m = __ballot(site);
                if (lane == 0) {
                    masks[c] = m;
                    carry[c] = last;
                }
                if (m)
                    last = c * 64 + 63 - __clzll(m);
                if (valid) {
                    const int64_t i = base + x;
                    if (MODE == 0) {
                        if (a.tq) a.tq[i] = kc[k];
                        if (a.tb1) a.tb1[i] = site ? 1 : 0;
                        if (a.tsb) a.tsb[i] = (int8_t)(site ? sgn : 0);
                    } else {
                        if (a.ts) a.ts[i] = (int8_t)kc[k];
                        if (a.td1) a.td1[i] = (wc[k] == QAI_WORD_INF) ? -1 : (int32_t)word_d2(wc[k]);
                        if (a.tb2) a.tb2[i] = site ? 1 : 0;
                    }
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        int next = -1; // first site after the current chunk
        for (int c = nch - 1; c >= 0; --c) {
            const uint64_t m = masks[c];
            const int cl = carry[c];
            const int64_t x = (int64_t)c * 64 + lane;
            const int hb = highest_at_or_below(m, lane);
            const int lb = lowest_at_or_above(m, lane);
            const int L = hb >= 0 ? c * 64 + hb : cl;
            const int R = lb >= 0 ? c * 64 + lb : next;
            uint32_t word = QAI_WORD_INF;
            if (L >= 0 || R >= 0) {
                const int dl = L >= 0 ? (int)x - L : 0x7fffffff;
                const int dr = R >= 0 ? R - (int)x : 0x7fffffff;
                const int s = (dl <= dr) ? L : R;
                const uint32_t d = (uint32_t)(dl <= dr ? dl : dr);
                const uint32_t code = (MODE == 0) ? (uint32_t)codes[s] : 0u;
                word = word_make(d * d, code);
            }
            if (x < nx)
                a.wout[base + x] = word;
            if (m)
                next = c * 64 + __ffsll((unsigned long long)m) - 1;
        }
        if (MODE == 0 && __ballot(bad) && lane == 0)
            atomicOr(a.status, QAI_STATUS_QRANGE);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// 2.5-D variant of the seed pass.  A workgroup owns Ty adjacent x-lines
// (one wave each) and marches along z over Tz planes; the stencil keys of
// rows y-1 .. y+Ty in planes z-1, z, z+1 live in an LDS ring of three planes,
// so every input word is loaded and converted once per block (plus the halo
// rows).  Keys: mode 0 the recovered index q; mode 1 the propagated sign S
// in bits 0-1 and the B1 flag in bit 2.  Each wave then marks its row's sites
// and runs the same ballot scan along x as k_seed_xscan.
struct SlabArgs {
    SeedArgs s;
    int ty, tz;         // rows (waves) per block, planes per block
    int rows, planes;   // ring rows (ty + 2, or 1 when ny == 1) and planes (3, or 1 when nz == 1)
    int64_t nby, nbz;   // blocks along y and z
};

template <int MODE>
__device__ __forceinline__ int slab_key(const SeedArgs& a, int64_t i, bool& bad)
{
    if (MODE == 0)
        return recover_q(a.xq[i], a.inv2eb, a.two_eb, bad);
    const uint32_t w = a.w1[i];
    const int sgn = word_sign(w);
    const int b1 = (w != QAI_WORD_INF && word_d2(w) == 0u) ? 4 : 0;
    return (sgn & 3) | b1;
}

template <int MODE>
__global__ __launch_bounds__(512) void k_seed_slab(SlabArgs A)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const SeedArgs& a = A.s;
    const int nx = (int)a.nx;
    const int64_t ny = a.ny, nz = a.nz;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nch = (nx + 63) >> 6;
    const size_t ring_bytes = ((size_t)A.planes * A.rows * nx * 4 + 15) & ~(size_t)15;
    int* ring = (int*)smem;                                       // [plane][row][x]
    unsigned char* tail = smem + ring_bytes;
    unsigned char* codes = tail + (size_t)wave * nch * 64;
    uint64_t* masks = (uint64_t*)(tail + (size_t)A.ty * nch * 64) + (size_t)wave * nch;
    int* carry = (int*)(tail + (size_t)A.ty * nch * 72) + (size_t)wave * nch;
    const int64_t plane = (int64_t)nx * ny;
    const bool hy = ny > 1, hz = nz > 1, hx = nx > 1;
    const uint64_t nblocks = (uint64_t)(A.nby * A.nbz);

    for (uint64_t t = blockIdx.x; t < nblocks; t += gridDim.x) {
        const uint64_t bl = xcd_remap(t, nblocks);
        const int64_t by = (int64_t)(bl % (uint64_t)A.nby), bz = (int64_t)(bl / (uint64_t)A.nby);
        const int64_t y0 = by * A.ty, z0 = bz * A.tz;
        const int64_t z1 = min(nz, z0 + A.tz);
        const int64_t ry0 = hy ? y0 - 1 : y0; // y of ring row 0
        bool bad = false;

        // stage plane zz into its ring slot (rows outside the domain read as 0)
        auto stage = [&](int64_t zz) {
            int* dst = ring + (int)((hz ? (zz + 3) % 3 : 0) * A.rows * nx);
            for (int r = 0; r < A.rows; ++r) {
                const int64_t yy = ry0 + r;
                const bool in = zz >= 0 && zz < nz && yy >= 0 && yy < ny;
                const int64_t rb = zz * plane + yy * nx;
                for (int x = threadIdx.x; x < nx; x += blockDim.x)
                    dst[r * nx + x] = in ? slab_key<MODE>(a, rb + x, bad) : 0;
            }
        };
        lds_barrier();
        if (hz)
            stage(z0 - 1);
        stage(z0);
        for (int64_t z = z0; z < z1; ++z) {
            if (hz)
                stage(z + 1);
            lds_barrier();
            const int64_t y = y0 + wave;
            if (wave < A.ty && y < ny) {
                const int rc = hy ? wave + 1 : 0;
                const int* pc = ring + (int)((hz ? z % 3 : 0) * A.rows * nx);
                const int* pm = hz ? ring + (int)(((z + 2) % 3) * A.rows * nx) : pc;
                const int* pp = hz ? ring + (int)(((z + 1) % 3) * A.rows * nx) : pc;
                const int* rowc = pc + rc * nx;
                const int* rowym = hy ? pc + (rc - 1) * nx : rowc;
                const int* rowyp = hy ? pc + (rc + 1) * nx : rowc;
                const int* rowzm = pm + rc * nx;
                const int* rowzp = pp + rc * nx;
                const bool line_in = (!hy || (y >= 1 && y <= ny - 2)) && (!hz || (z >= 1 && z <= nz - 2));
                const int64_t base = (z * ny + y) * nx;
                int last = -1;
                for (int c = 0; c < nch; ++c) {
                    const int x = c * 64 + lane;
                    const bool valid = x < nx;
                    const int kc = valid ? rowc[x] : 0;
                    const bool x_in = !hx || (x >= 1 && x <= nx - 2);
                    bool site = false;
                    int sgn = 0;
                    if (valid && line_in && x_in) {
                        const int kp = hx ? rowc[x + 1] : kc, km = hx ? rowc[x - 1] : kc;
                        const int ky1 = rowyp[x], ky0 = rowym[x], kz1 = rowzp[x], kz0 = rowzm[x];
                        if (MODE == 0) {
                            // Algorithm 2: boundary if some 6-neighbour index differs; sign of the
                            // first differing neighbour (+x, -x, +y, -y, +z, -z); discarded where
                            // an absolute central difference reaches 1 (|q+ - q-| >= 2).
                            int first = (kp != kc) ? kp - kc : ((km != kc) ? km - kc : 0);
                            if (first == 0)
                                first = (ky1 != kc) ? ky1 - kc : ((ky0 != kc) ? ky0 - kc : 0);
                            if (first == 0)
                                first = (kz1 != kc) ? kz1 - kc : ((kz0 != kc) ? kz0 - kc : 0);
                            const bool steep = abs(kp - km) >= 2 || abs(ky1 - ky0) >= 2 || abs(kz1 - kz0) >= 2;
                            if (first != 0) {
                                site = true;
                                sgn = steep ? 0 : (first > 0 ? 1 : -1);
                            }
                        } else {
                            // Algorithm 3's GetBoundary(S): interior voxels outside B1 whose
                            // propagated sign differs from a 6-neighbour's.
                            const int sc = kc & 3;
                            site = !(kc & 4) && (((kp & 3) != sc) || ((km & 3) != sc) || ((ky1 & 3) != sc) ||
                                                 ((ky0 & 3) != sc) || ((kz1 & 3) != sc) || ((kz0 & 3) != sc));
                        }
                    }
                    if (MODE == 0)
                        codes[c * 64 + lane] = (unsigned char)sign_code(sgn);
                    const uint64_t m = __ballot(site);
                    if (lane == 0) {
                        masks[c] = m;
                        carry[c] = last;
                    }
                    if (m)
                        last = c * 64 + 63 - __clzll(m);
                    if (valid) {
                        const int64_t i = base + x;
                        if (MODE == 0) {
                            if (a.tq) a.tq[i] = kc;
                            if (a.tb1) a.tb1[i] = site ? 1 : 0;
                            if (a.tsb) a.tsb[i] = (int8_t)(site ? sgn : 0);
                        } else {
                            const int sg = (kc & 3) == 1 ? 1 : ((kc & 3) == 3 ? -1 : 0);
                            if (a.ts) a.ts[i] = (int8_t)sg;
                            if (a.td1) {
                                const uint32_t w = a.w1[i];
                                a.td1[i] = (w == QAI_WORD_INF) ? -1 : (int32_t)word_d2(w);
                            }
                            if (a.tb2) a.tb2[i] = site ? 1 : 0;
                        }
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                int next = -1;
                for (int c = nch - 1; c >= 0; --c) {
                    const uint64_t m = masks[c];
                    const int cl = carry[c];
                    const int x = c * 64 + lane;
                    const int hb = highest_at_or_below(m, lane);
                    const int lb = lowest_at_or_above(m, lane);
                    const int L = hb >= 0 ? c * 64 + hb : cl;
                    const int R = lb >= 0 ? c * 64 + lb : next;
                    uint32_t word = QAI_WORD_INF;
                    if (L >= 0 || R >= 0) {
                        const int dl = L >= 0 ? x - L : 0x7fffffff;
                        const int dr = R >= 0 ? R - x : 0x7fffffff;
                        const int st = (dl <= dr) ? L : R;
                        const uint32_t d = (uint32_t)(dl <= dr ? dl : dr);
                        const uint32_t code = (MODE == 0) ? (uint32_t)codes[st] : 0u;
                        word = word_make(d * d, code);
                    }
                    if (x < nx)
                        a.wout[base + x] = word;
                    if (m)
                        next = c * 64 + __ffsll((unsigned long long)m) - 1;
                }
            }
            lds_barrier();
        }
        if (MODE == 0 && __ballot(bad) && lane == 0)
            atomicOr(a.status, QAI_STATUS_QRANGE);
    }
}

// Long x-lines (more than 512 voxels): one line per workgroup, its chunks of
// 64 voxels split between the SEG wavefronts, so that a line's two sweeps
// run in parallel pieces instead of one wave walking the whole line.  Sweep 1
// (each wave over its own chunks): stencil and sites as k_seed_slab, the
// chunk's site mask and codes, and the last site before each chunk within the
// wave's piece.  After a barrier each wave takes the last site left of its
// piece and the first one right of it from the other pieces' masks, then runs
// sweep 2 over its chunks.  The ring holds the line and its two neighbour
// lines of planes z-1, z, z+1; the block marches tz planes.
template <int MODE, int SEG>
__global__ __launch_bounds__(64 * SEG) void k_seed_seg(SlabArgs A)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const SeedArgs& a = A.s;
    const int nx = (int)a.nx;
    const int64_t ny = a.ny, nz = a.nz;
    const int wave = (int)(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int nch = (nx + 63) >> 6;
    const int c0 = (wave * nch) / SEG, c1 = ((wave + 1) * nch) / SEG;   // this wave's chunks
    const size_t ring_bytes = ((size_t)A.planes * A.rows * nx * 4 + 15) & ~(size_t)15;
    int* ring = (int*)smem;                                              // [plane][row][x]
    unsigned char* codes = smem + ring_bytes;                            // [chunk][lane]
    uint64_t* masks = (uint64_t*)(codes + (((size_t)nch * 64 + 15) & ~(size_t)15));
    int* lastb = (int*)(masks + nch);                                    // last site before chunk, in the piece
    const int64_t plane = (int64_t)nx * ny;
    const bool hy = ny > 1, hz = nz > 1, hx = nx > 1;
    const uint64_t nblocks = (uint64_t)(A.nby * A.nbz);

    for (uint64_t t = blockIdx.x; t < nblocks; t += gridDim.x) {
        const uint64_t bl = xcd_remap(t, nblocks);
        const int64_t y = (int64_t)(bl % (uint64_t)A.nby), bz = (int64_t)(bl / (uint64_t)A.nby);
        const int64_t z0 = bz * A.tz, z1 = min(nz, z0 + A.tz);
        const int64_t ry0 = hy ? y - 1 : y; // y of ring row 0
        bool bad = false;

        auto stage = [&](int64_t zz) {
            int* dst = ring + (int)((hz ? (zz + 3) % 3 : 0) * A.rows * nx);
            for (int r = 0; r < A.rows; ++r) {
                const int64_t yy = ry0 + r;
                const bool in = zz >= 0 && zz < nz && yy >= 0 && yy < ny;
                const int64_t rb = zz * plane + yy * nx;
                for (int x = threadIdx.x; x < nx; x += blockDim.x)
                    dst[r * nx + x] = in ? slab_key<MODE>(a, rb + x, bad) : 0;
            }
        };
        lds_barrier();
        if (hz)
            stage(z0 - 1);
        stage(z0);
        for (int64_t z = z0; z < z1; ++z) {
            if (hz)
                stage(z + 1);
            lds_barrier();
            const int rc = hy ? 1 : 0;
            const int* pc = ring + (int)((hz ? z % 3 : 0) * A.rows * nx);
            const int* pm = hz ? ring + (int)(((z + 2) % 3) * A.rows * nx) : pc;
            const int* pp = hz ? ring + (int)(((z + 1) % 3) * A.rows * nx) : pc;
            const int* rowc = pc + rc * nx;
            const int* rowym = hy ? pc + (rc - 1) * nx : rowc;
            const int* rowyp = hy ? pc + (rc + 1) * nx : rowc;
            const int* rowzm = pm + rc * nx;
            const int* rowzp = pp + rc * nx;
            const bool line_in = (!hy || (y >= 1 && y <= ny - 2)) && (!hz || (z >= 1 && z <= nz - 2));
            const int64_t base = (z * ny + y) * nx;
            // sweep 1 over this wave's chunks
            int last = -1;
            for (int c = c0; c < c1; ++c) {
                const int x = c * 64 + lane;
                const bool valid = x < nx;
                const int kc = valid ? rowc[x] : 0;
                const bool x_in = !hx || (x >= 1 && x <= nx - 2);
                bool site = false;
                int sgn = 0;
                if (valid && line_in && x_in) {
                    const int kp = hx ? rowc[x + 1] : kc, km = hx ? rowc[x - 1] : kc;
                    const int ky1 = rowyp[x], ky0 = rowym[x], kz1 = rowzp[x], kz0 = rowzm[x];
                    if (MODE == 0) {
                        // Algorithm 2 (as in k_seed_slab)
                        int first = (kp != kc) ? kp - kc : ((km != kc) ? km - kc : 0);
                        if (first == 0)
                            first = (ky1 != kc) ? ky1 - kc : ((ky0 != kc) ? ky0 - kc : 0);
                        if (first == 0)
                            first = (kz1 != kc) ? kz1 - kc : ((kz0 != kc) ? kz0 - kc : 0);
                        const bool steep = abs(kp - km) >= 2 || abs(ky1 - ky0) >= 2 || abs(kz1 - kz0) >= 2;
                        if (first != 0) {
                            site = true;
                            sgn = steep ? 0 : (first > 0 ? 1 : -1);
                        }
                    } else {
                        // Algorithm 3's GetBoundary(S) (as in k_seed_slab)
                        const int sc = kc & 3;
                        site = !(kc & 4) && (((kp & 3) != sc) || ((km & 3) != sc) || ((ky1 & 3) != sc) ||
                                             ((ky0 & 3) != sc) || ((kz1 & 3) != sc) || ((kz0 & 3) != sc));
                    }
                }
                if (MODE == 0)
                    codes[c * 64 + lane] = (unsigned char)sign_code(sgn);
                const uint64_t m = __ballot(site);
                if (lane == 0) {
                    masks[c] = m;
                    lastb[c] = last;
                }
                if (m)
                    last = c * 64 + 63 - __clzll(m);
                if (valid) {
                    const int64_t i = base + x;
                    if (MODE == 0) {
                        if (a.tq) a.tq[i] = kc;
                        if (a.tb1) a.tb1[i] = site ? 1 : 0;
                        if (a.tsb) a.tsb[i] = (int8_t)(site ? sgn : 0);
                    } else {
                        const int sg = (kc & 3) == 1 ? 1 : ((kc & 3) == 3 ? -1 : 0);
                        if (a.ts) a.ts[i] = (int8_t)sg;
                        if (a.td1) {
                            const uint32_t w = a.w1[i];
                            a.td1[i] = (w == QAI_WORD_INF) ? -1 : (int32_t)word_d2(w);
                        }
                        if (a.tb2) a.tb2[i] = site ? 1 : 0;
                    }
                }
            }
            lds_barrier();
            // the nearest sites outside this wave's piece
            int carry_l = -1, carry_r = -1;
            for (int c = c0 - 1; c >= 0; --c) {
                const uint64_t m = masks[c];
                if (m) {
                    carry_l = c * 64 + 63 - __clzll(m);
                    break;
                }
            }
            for (int c = c1; c < nch; ++c) {
                const uint64_t m = masks[c];
                if (m) {
                    carry_r = c * 64 + __ffsll((unsigned long long)m) - 1;
                    break;
                }
            }
            // sweep 2 over this wave's chunks: nearest of the two, ties to the left site
            int next = carry_r;
            for (int c = c1 - 1; c >= c0; --c) {
                const uint64_t m = masks[c];
                const int lbc = lastb[c];
                const int cl = lbc >= 0 ? lbc : carry_l;
                const int x = c * 64 + lane;
                const int hb = highest_at_or_below(m, lane);
                const int lb = lowest_at_or_above(m, lane);
                const int L = hb >= 0 ? c * 64 + hb : cl;
                const int R = lb >= 0 ? c * 64 + lb : next;
                uint32_t word = QAI_WORD_INF;
                if (L >= 0 || R >= 0) {
                    const int dl = L >= 0 ? x - L : 0x7fffffff;
                    const int dr = R >= 0 ? R - x : 0x7fffffff;
                    const int st = (dl <= dr) ? L : R;
                    const uint32_t d = (uint32_t)(dl <= dr ? dl : dr);
                    const uint32_t code = (MODE == 0) ? (uint32_t)codes[st] : 0u;
                    word = word_make(d * d, code);
                }
                if (x < nx)
                    a.wout[base + x] = word;
                if (m)
                    next = c * 64 + __ffsll((unsigned long long)m) - 1;
            }
            lds_barrier();
        }
        if (MODE == 0 && __ballot(bad) && lane == 0)
            atomicOr(a.status, QAI_STATUS_QRANGE);
    }
}

__device__ __forceinline__ int32_t raw_word_d1(const uint32_t* w1, int64_t i)
{
    const uint32_t w = w1[i];
    return (w == QAI_WORD_INF) ? -1 : (int32_t)word_d2(w);
}

// Seed passes for lines of up to 64 * V voxels, lane l of a wave owning voxels
// [V l, V l + V) of its line.  A workgroup of WPB wavefronts owns WPB adjacent
// x-lines (one per wave) and marches them through tz planes.  Each wave keeps
// its own line of planes z-1, z, z+1 in registers (the +-z neighbours); the
// current plane's lines of the group and its two halo lines sit in LDS (the
// +-y neighbours; double-buffered, one barrier per plane).  The +-x neighbours
// are the lane's own registers except at its two ends.  The x pass of the EDT
// needs no per-voxel masks: each lane scans its own voxels in order (nearest
// site at or before, at or after) and takes one carry per direction from the
// nearest lane holding a site.  Lines are
// read and written VW words per access (VW divides V and nx).  LDS lines are
// lane-major: voxel V l + j at j * 64 + l, so every LDS access of a wave is
// 64 consecutive words.
// Lines of more than 512 voxels (P > 1): P waves share a line, wave p owning
// its piece [512 p, 512 p + 512) (V = 8); the +-x neighbours across a piece's
// ends come from the LDS line, and the x pass's carries from the other pieces
// from a per-plane exchange of each piece's first and last site (a second
// barrier per plane).
template <int MODE, int V, int WPB, int VW, bool TAPS, int P = 1>
__global__ __launch_bounds__(64 * WPB) void k_seed_lane(SlabArgs A)
{
    static_assert(V % VW == 0, "vector width must divide the voxels per lane");
    static_assert(P == 1 || (V == 8 && WPB % P == 0 && WPB / P >= 2), "pieces of 512 voxels, two lines or more per workgroup");
    // MODE 0: step A from the decompressed field; 2: step A from coded
    // indices (decoded here, x' = 2 eb q written to xout); 1: step C
    constexpr bool SA = MODE != 1, CODED = MODE == 2;
    static_assert(!CODED || (32 % V == 0 && !TAPS), "coded input: a lane's voxels lie in one 32-voxel segment");
    constexpr int PW = V * 64;     // voxels of a wave's piece of its line
    constexpr int W = PW * P;      // LDS words per line
    constexpr int LP = WPB / P;    // lines per workgroup
    constexpr int R = LP + 2;
    __shared__ uint32_t rows[2][R * W];
    __shared__ uint32_t pinfo[P > 1 ? LP * P * 2 : 1]; // per piece: last site, first site
    __shared__ unsigned long long b1sum;
    const SeedArgs& a = A.s;
    const int nx = (int)a.nx;
    const int64_t ny = a.ny, nz = a.nz;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int line = wave / P, piece = wave % P;
    const bool hy = ny > 1, hz = nz > 1, hx = nx > 1;
    const uint32_t* __restrict__ src = (SA) ? (const uint32_t*)a.xq : a.w1;
    const int x0 = piece * PW + V * lane;  // first voxel of the lane
    const int cs = CODED ? min(x0 >> 5, (int)a.segs_row - 1) : 0;
    const int cp0 = x0 - (cs << 5);
    const __amdgpu_buffer_rsrc_t prs = payload_rsrc(CODED ? a.cpay : nullptr, CODED ? a.cpay_bytes : 0u);
    // stencil range along x: the interior when the axis exists
    const int xmax = hx ? nx - 2 : nx - 1;
    const bool first_in = x0 >= (hx ? 1 : 0);
    const uint64_t lower = (1ull << lane) - 1ull;                        // lanes strictly below
    const uint64_t upper = (lane == 63) ? 0ull : (~0ull << (lane + 1));  // strictly above
    const uint64_t nblocks = (uint64_t)(A.nby * A.nbz);
    bool bad = false;
    uint32_t nb1 = 0u; // mode 0: B1 among the lanes' first voxels, a 1-in-V sample (wave-uniform)
    if (SA && a.b1count) {
        if (threadIdx.x == 0)
            b1sum = 0ull;
        lds_barrier();
    }

    // Site value of voxel x with payload code: ((x + 4096) << 2) | code, so
    // values order like positions.  "No site" to the left is 0, to the right
    // NONE_R; either lies more than 4096 voxels away.
    constexpr uint32_t NONE_R = (8191u + 4096u) << 2;

    for (uint64_t t = blockIdx.x; t < nblocks; t += gridDim.x) {
        const uint64_t bl = xcd_remap(t, nblocks);
        const int64_t by = (int64_t)(bl % (uint64_t)A.nby), bz = (int64_t)(bl / (uint64_t)A.nby);
        const int64_t y0 = by * LP, z0 = bz * A.tz;
        const int64_t z1 = min(nz, z0 + A.tz);
        const int64_t y = y0 + line;
        const int64_t yh = (line == 0) ? y0 - 1 : y0 + LP;
        const bool halo = hy && (line == 0 || line == LP - 1);
        const int hrow = (line == 0) ? 0 : R - 1;

        // Coded input: a line's decode in flight -- its segment head, the
        // payload words of the lane's share, whether the line lies in the field.
        // The lane's share of its row: segment cs = x0 / 32 (lanes past the
        // row's end take the last segment; their values are not used), voxels
        // [cp0, cp0 + V) of it; the 32 / V lanes of a segment are consecutive.
        struct Pend {
            CodeHead h;
            uint32_t w4[4];
            bool ok;
        };
        auto seg_of = [&](int64_t zz, int64_t yy, bool ok) -> int64_t {
            return ((ok ? zz : 0) * ny + (ok ? yy : 0)) * a.segs_row + cs;
        };
        // step one: the segment head (meta word and first index)
        auto start = [&](int64_t zz, int64_t yy) -> Pend {
            Pend pd;
            pd.ok = zz >= 0 && zz < nz && yy >= 0 && yy < ny;
            pd.h = code_head(a.cbase, a.cmeta, seg_of(zz, yy, pd.ok));
            return pd;
        };
        // step two: the payload words
        auto fetch = [&](Pend& pd) { code_words<V>(prs, pd.h, cp0, pd.w4); };
        // Loads go to valid addresses without branching: a line outside the
        // field reads line 0 and a group of words past the end of the line the
        // line's first group; keys() substitutes 0 for them (nx is a multiple
        // of VW: a group lies wholly inside or outside).  A branch here would
        // leave the loaded registers to merge with zeros at its join, and the
        // copy there waits for the loads: the prefetch would be lost.
        auto load = [&](int64_t zz, int64_t yy, uint32_t (&r)[V]) -> bool {
            const bool ok = zz >= 0 && zz < nz && yy >= 0 && yy < ny;
            if constexpr (CODED) {
                // the lane's V indices of the line, decoded at once (the
                // prologue); the plane loop pipelines the steps (Pend)
                Pend pd = start(zz, yy);
                fetch(pd);
                int32_t qv[V];
                code_finish<V>(prs, pd.h, pd.w4, cp0, lane, qv);
#pragma unroll
                for (int j = 0; j < V; ++j)
                    r[j] = (uint32_t)qv[j];
                return pd.ok;
            }
            const uint32_t* p = src + ((ok ? zz : 0) * ny + (ok ? yy : 0)) * (int64_t)nx;
#pragma unroll
            for (int j = 0; j < V; j += VW) {
                const uint32_t* q = p + (x0 + j < nx ? x0 + j : 0);
                if (VW == 4) {
                    const uint4 v = *(const uint4*)q;
                    r[j] = v.x, r[j + 1] = v.y, r[j + 2] = v.z, r[j + 3] = v.w;
                } else if (VW == 2) {
                    const uint2 v = *(const uint2*)q;
                    r[j] = v.x, r[j + 1] = v.y;
                } else {
                    r[j] = *q;
                }
            }
            return ok;
        };
        // Keys: mode 0 the quantization index with its sign bit flipped (the
        // unsigned order of the keys is then the signed order of q); mode 1
        // the sign code of the first-EDT word (0: S = 0, 1: +1, 2: -1; 3 for
        // "no site", which occurs only when B1 is empty, everywhere at once)
        // plus 4 on B1 (distance 0).
        auto keys = [&](const uint32_t (&r)[V], bool ok, uint32_t (&k)[V]) {
            if constexpr (SA && !CODED) {
                // recover_q's fast case (the product with the rounded
                // reciprocal within 0.4 of an integer below 2^18) tested for
                // the lane's V voxels together; only a wave where some voxel
                // fails it takes recover_q voxel by voxel
                float t[V], rt[V];
                float dev = 0.0f, mag = 0.0f;
#pragma unroll
                for (int j = 0; j < V; ++j) {
                    const bool in = ok && x0 + j < nx;
                    t[j] = (in ? __uint_as_float(r[j]) : 0.0f) * a.inv2eb;
                    rt[j] = rintf(t[j]);
                    dev = fmaxf(dev, fabsf(t[j] - rt[j]));
                    mag = fmaxf(mag, fabsf(t[j]));
                }
                // (a NaN compares false: such a lane takes the voxel-wise path)
                if (__ballot(!(mag < 262144.0f && dev <= 0.4f)) == 0ull) {
#pragma unroll
                    for (int j = 0; j < V; ++j)
                        k[j] = (uint32_t)(int32_t)rt[j] ^ 0x80000000u;
                    return;
                }
            }
#pragma unroll
            for (int j = 0; j < V; ++j) {
                const bool in = ok && x0 + j < nx;
                const uint32_t w = in ? r[j] : 0u;
                if (CODED) {
                    const int32_t qv = (int32_t)w;
                    bad = bad || qv > (1 << 21) || qv < -(1 << 21);
                    k[j] = w ^ 0x80000000u;
                } else if (SA)
                    k[j] = (uint32_t)recover_q(__uint_as_float(w), a.inv2eb, a.two_eb, bad) ^ 0x80000000u;
                else
                    k[j] = (w & 3u) | (w < 4u ? 4u : 0u);
            }
        };
        auto put = [&](int b, int row, const uint32_t (&k)[V]) {
#pragma unroll
            for (int j = 0; j < V; ++j)
                rows[b][row * W + piece * PW + j * 64 + lane] = k[j];
        };

        uint32_t raw[V], hraw[V];
        uint32_t P0[V], P1[V], P2[V];
        bool rok = load(z0 - 1, y, raw), hok = false;
        keys(raw, rok, P0);
        rok = load(z0, y, raw);
        keys(raw, rok, P1);
        if (halo)
            hok = load(z0, yh, hraw);
        rok = load(z0 + 1, y, raw);
        keys(raw, rok, P2);
        if (!hz) {
            // a flat z axis: the +-z neighbours are the voxel itself
#pragma unroll
            for (int j = 0; j < V; ++j)
                P0[j] = P2[j] = P1[j];
        }
        lds_barrier();
        put(0, line + 1, P1);
        if (halo) {
            uint32_t H[V];
            keys(hraw, hok, H);
            put(0, hrow, H);
        }
        // coded input, decodes in flight: the segment heads of own line z0 + 2
        // and halo line z0 + 1 requested (the plane loop keeps this shape and
        // requests a line's payload words when it decodes the line)
        Pend po{}, ph{};
        if constexpr (CODED) {
            po = start(z0 + 2, y);
            if (halo)
                ph = start(z0 + 1, yh);
        } else {
            rok = load(z0 + 2, y, raw);
            if (halo)
                hok = load(z0 + 1, yh, hraw);
        }
        lds_barrier();

        int cur = 0;
        for (int64_t z = z0; z < z1; ++z) {
            // (pieces of longer lines: every wave takes part, for the barrier
            // of the site exchange; a line past the field's end stores nothing)
            if (P > 1 || y < ny) {
                const bool act = y < ny;
                if (CODED && act) {
                    // the decompressed value of the wave's own line, x' = 2 eb q
                    // (the exact product rounded once: the decompressor's value)
                    float* const xrow = a.xout + (z * ny + y) * (int64_t)nx + x0;
#pragma unroll
                    for (int j = 0; j < V; j += VW) {
                        if (x0 + j < nx) {
                            float xv[VW];
#pragma unroll
                            for (int u = 0; u < VW; ++u)
                                xv[u] = (float)(int32_t)(P1[j + u] ^ 0x80000000u) * a.two_eb;
                            if constexpr (VW == 4)
                                *(float4*)(xrow + j) = make_float4(xv[0], xv[1], xv[2], xv[3]);
                            else if constexpr (VW == 2)
                                *(float2*)(xrow + j) = make_float2(xv[0], xv[1]);
                            else
                                xrow[j] = xv[0];
                        }
                    }
                }
                const uint32_t* rc = &rows[cur][(line + 1) * W + piece * PW];
                const uint32_t* rym = hy ? rc - W : rc;
                const uint32_t* ryp = hy ? rc + W : rc;
                const bool line_in = (!hy || (y >= 1 && y <= ny - 2)) && (!hz || (z >= 1 && z <= nz - 2));
                // the neighbours across the lane's two ends (a flat x axis: itself)
                // (a piece of a longer line: across its ends, the neighbouring
                // pieces' end voxels)
                uint32_t kleft = P1[0], kright = P1[V - 1];
                if (hx) {
                    if constexpr (P == 1) {
                        kleft = rc[(V - 1) * 64 + (lane > 0 ? lane - 1 : 0)];
                        kright = rc[lane < 63 ? lane + 1 : 63];
                    } else {
                        kleft = rc[lane > 0 ? (V - 1) * 64 + lane - 1 : (piece > 0 ? -1 : (V - 1) * 64)];
                        kright = rc[lane < 63 ? lane + 1 : (piece < P - 1 ? PW : 63)];
                    }
                }
                bool st[V];      // voxel x0 + j is a site
                uint32_t sv[V];  // its site value
#pragma unroll
                for (int j = 0; j < V; ++j) {
                    const int x = x0 + j;
                    const uint32_t kc = P1[j];
                    const uint32_t kxp = j + 1 < V ? P1[j + 1] : kright;
                    const uint32_t kxm = j > 0 ? P1[j - 1] : kleft;
                    const uint32_t kyp = ryp[j * 64 + lane], kym = rym[j * 64 + lane];
                    const uint32_t kzp = P2[j], kzm = P0[j];
                    const bool in = act && line_in && x <= xmax && (j > 0 || first_in);
                    uint32_t code = 0u;
                    if (SA) {
                        // Algorithm 2 (see k_seed_slab): g is the first neighbour that
                        // differs from the voxel, in the order +x, -x, +y, -y, +z, -z
                        uint32_t g = (kxp != kc) ? kxp : kxm;
                        g = (g != kc) ? g : ((kyp != kc) ? kyp : kym);
                        g = (g != kc) ? g : ((kzp != kc) ? kzp : kzm);
                        // some axis differs by 2 or more: kp - km is not in {-1, 0, 1},
                        // i.e. kp - km + 1 (mod 2^32) exceeds 2
                        const bool steep = (kxp - kxm + 1u > 2u) | (kyp - kym + 1u > 2u) | (kzp - kzm + 1u > 2u);
                        st[j] = in && g != kc;
                        code = steep ? 0u : (g > kc ? 1u : 2u);
                        if (TAPS && act && x < nx) {
                            const int64_t i = (z * ny + y) * (int64_t)nx + x;
                            const int sgn = st[j] ? (code == 1u ? 1 : (code == 2u ? -1 : 0)) : 0;
                            if (a.tq) a.tq[i] = (int32_t)(kc ^ 0x80000000u);
                            if (a.tb1) a.tb1[i] = st[j] ? 1 : 0;
                            if (a.tsb) a.tsb[i] = (int8_t)sgn;
                        }
                    } else {
                        // Algorithm 3's GetBoundary(S) (see k_seed_slab)
                        const uint32_t diff = (kxp ^ kc) | (kxm ^ kc) | (kyp ^ kc) | (kym ^ kc) | (kzp ^ kc) | (kzm ^ kc);
                        st[j] = in && !(kc & 4u) && (diff & 3u) != 0u;
                        if (TAPS && act && x < nx) {
                            const int64_t i = (z * ny + y) * (int64_t)nx + x;
                            if (a.ts) a.ts[i] = (int8_t)((kc & 3u) == 1u ? 1 : ((kc & 3u) == 2u ? -1 : 0));
                            if (a.td1) a.td1[i] = raw_word_d1(a.w1, i);
                            if (a.tb2) a.tb2[i] = st[j] ? 1 : 0;
                        }
                    }
                    sv[j] = ((uint32_t)(x + 4096) << 2) | code;
                    if (SA && j == 0)
                        nb1 += (uint32_t)__popcll(__ballot(st[0]));
                }
                // nearest site at or before / at or after each voxel among the
                // lane's own
                uint32_t lv[V], rv[V];
                uint32_t L = 0u, Rr = NONE_R;
#pragma unroll
                for (int j = 0; j < V; ++j) {
                    L = st[j] ? sv[j] : L;
                    lv[j] = L;
                }
#pragma unroll
                for (int j = V - 1; j >= 0; --j) {
                    Rr = st[j] ? sv[j] : Rr;
                    rv[j] = Rr;
                }
                const uint64_t m = __ballot(lv[V - 1] != 0u);
                // nearest sites past the piece's ends (none for a whole line):
                // each piece posts its last and first site, then reads the others'
                uint32_t pl = 0u, pr = NONE_R;
                if constexpr (P > 1) {
                    const uint32_t last = (uint32_t)__shfl((int)lv[V - 1], m ? 63 - __clzll(m) : 0);
                    const uint32_t first = (uint32_t)__shfl((int)rv[0], m ? __ffsll((unsigned long long)m) - 1 : 0);
                    if (lane == 0) {
                        pinfo[(line * P + piece) * 2] = m ? last : 0u;
                        pinfo[(line * P + piece) * 2 + 1] = m ? first : NONE_R;
                    }
                    lds_barrier();
#pragma unroll
                    for (int q = 0; q < P; ++q) {
                        if (q < piece)
                            pl = max(pl, pinfo[(line * P + q) * 2]);
                        if (q > piece)
                            pr = min(pr, pinfo[(line * P + q) * 2 + 1]);
                    }
                }
                // the carries: the last site of the nearest lane below holding
                // one, the first of the nearest lane above (a value from below is
                // smaller than any own one, from above larger), else pl / pr
                const uint64_t ml = m & lower, mr = m & upper;
                const int sl = ml ? 63 - __clzll(ml) : 0;
                const int sr = mr ? __ffsll((unsigned long long)mr) - 1 : 0;
                const uint32_t cl = (uint32_t)__shfl((int)lv[V - 1], sl);
                const uint32_t cr = (uint32_t)__shfl((int)rv[0], sr);
                const uint32_t carry_l = ml ? cl : pl, carry_r = mr ? cr : pr;
                uint32_t word[V];
#pragma unroll
                for (int j = 0; j < V; ++j) {
                    // sweep result: nearest of the two, ties to the left site;
                    // distances in units of 4 (d4 = 4 d, d4^2 / 4 = d^2 << 2)
                    const uint32_t Lj = max(lv[j], carry_l), Rj = min(rv[j], carry_r);
                    const uint32_t xb4 = (uint32_t)(x0 + j + 4096) << 2;
                    const uint32_t cm = (SA) ? ~3u : ~0u; // mode 1 values carry no code
                    const uint32_t dl4 = xb4 - (Lj & cm), dr4 = (Rj & cm) - xb4;
                    const bool left = dl4 <= dr4;
                    const uint32_t d4 = left ? dl4 : dr4;
                    const uint32_t cd = (SA) ? ((left ? Lj : Rj) & 3u) : 0u;
                    word[j] = (__umul24(d4, d4) >> 2) | cd;
                }
                if (m == 0ull && pl == 0u && pr == NONE_R) {
                    // no site on the line
#pragma unroll
                    for (int j = 0; j < V; ++j)
                        word[j] = QAI_WORD_INF;
                }
                if (act) {
                    uint32_t* const wrow = a.wout + (z * ny + y) * (int64_t)nx + x0;
#pragma unroll
                    for (int j = 0; j < V; j += VW) {
                        if (x0 + j < nx) {
                            if (VW == 4)
                                *(uint4*)(wrow + j) = make_uint4(word[j], word[j + 1], word[j + 2], word[j + 3]);
                            else if (VW == 2)
                                *(uint2*)(wrow + j) = make_uint2(word[j], word[j + 1]);
                            else
                                wrow[j] = word[j];
                        }
                    }
                }
            }
            if (z + 1 < z1) {
#pragma unroll
                for (int j = 0; j < V; ++j) {
                    P0[j] = P1[j];
                    P1[j] = P2[j];
                }
                if constexpr (CODED) {
                    int32_t qv[V];
                    fetch(po);
                    if (halo)
                        fetch(ph);
                    code_finish<V>(prs, po.h, po.w4, cp0, lane, qv);
#pragma unroll
                    for (int j = 0; j < V; ++j)
                        raw[j] = (uint32_t)qv[j];
                    rok = po.ok;
                    if (halo) {
                        code_finish<V>(prs, ph.h, ph.w4, cp0, lane, qv);
#pragma unroll
                        for (int j = 0; j < V; ++j)
                            hraw[j] = (uint32_t)qv[j];
                        hok = ph.ok;
                    }
                }
                keys(raw, rok, P2);
                put(cur ^ 1, line + 1, P1);
                if (halo) {
                    uint32_t H[V];
                    keys(hraw, hok, H);
                    put(cur ^ 1, hrow, H);
                }
                if constexpr (CODED) {
                    po = start(z + 3, y);
                    if (halo)
                        ph = start(z + 2, yh);
                } else {
                    rok = load(z + 3, y, raw);
                    if (halo)
                        hok = load(z + 2, yh, hraw);
                }
            }
            lds_barrier();
            cur ^= 1;
        }
    }
    if (SA && __ballot(bad) && (threadIdx.x & 63) == 0)
        atomicOr(a.status, QAI_STATUS_QRANGE);
    if (SA && a.b1count) {
        if ((threadIdx.x & 63) == 0)
            atomicAdd(&b1sum, (unsigned long long)nb1 * V);
        lds_barrier();
        if (threadIdx.x == 0)
            atomicAdd(a.b1count, b1sum);
    }
}

// ---------------------------------------------------------- interpolation
// Step E for one voxel: C = w * S * eta * eb, out = x' + C (x' copied as is
// where S = 0).
__device__ __forceinline__ void interp_store(int64_t i, uint32_t w2word, const uint32_t* __restrict__ w1,
                                             const float* xq, float* out, float eta_eb, float power,
                                             int32_t* td2, float* tw)
{
    const uint32_t w1word = w1[i];
    const int s = word_sign(w1word);
    const float xv = xq[i];
    const bool none2 = (w2word == QAI_WORD_INF);
    const bool none1 = (w1word == QAI_WORD_INF);
    const float wt = idw_weight(none1 ? 0u : word_d2(w1word), none1, none2 ? 0u : word_d2(w2word), none2, power);
    out[i] = (s == 0) ? xv : fmaf(wt, (float)s * eta_eb, xv);
    if (td2)
        td2[i] = none2 ? -1 : (int32_t)word_d2(w2word);
    if (tw)
        tw[i] = wt;
}

// Where B1 covers less than 60% of the field (the first seed pass's
// estimate) most voxels need d2 (on 128x128x1024 and 100x500x500 fields at
// rel. bounds 4e-3..1e-2: 48-81%), and a whole z pass with step E beats the
// needed-voxel search (0.66-0.98 against 0.98-1.39 ms; at 93% B1 the search
// wins, 0.65 against 0.76 ms).  The two are launched side by side, each gated
// on this test.
__device__ __forceinline__ bool sparse_b1(const unsigned long long* b1count, uint64_t n)
{
    return *b1count * 5ull < n * 3ull;
}

// With only_sparse set the kernel finishes what the needed-voxel search
// would: voxels with S != 0 off B1 and off B2 (w2 != 0), whose out the
// streaming phase left at x' (so x' may alias out); every other voxel keeps
// the streaming phase's value.
__global__ __launch_bounds__(256) void k_interp(InterpArgs a)
{
    if (a.only_sparse) {
        if (!sparse_b1(a.only_sparse, (uint64_t)a.n))
            return;
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * blockDim.x) {
            const uint32_t w1w = a.w1[i];
            if (word_sign(w1w) == 0 || w1w == QAI_WORD_INF || word_d2(w1w) == 0u)
                continue;
            const uint32_t w2w = a.w2[i];
            if (w2w != 0u)
                interp_store(i, w2w, a.w1, a.xq, a.out, a.eta_eb, a.power, nullptr, nullptr);
        }
        return;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * blockDim.x)
        interp_store(i, a.w2[i], a.w1, a.xq, a.out, a.eta_eb, a.power, a.td2, a.tw);
}

// Step E over a 3-D field with the last pass of step D done only where the
// weight needs the distance to B2: S != 0 off B1 ("needed" voxels).  There
// d2 = min over z' of G(z') + (z - z')^2 with G the result of the y pass;
// everywhere else out = x' (S = 0) or x' + S eta eb (on B1), exactly as
// interp_store computes them.  Two phases:
//   k_interp_own   streams w1 and x' (four voxels per thread, 16-byte
//                  accesses) and writes out.  At a needed voxel it reads
//                  G(z) itself: G(z) = 0 means the voxel is on B2 (w = 0) and
//                  is finished; otherwise out keeps x' for now and the voxel
//                  is flagged: per wave, four 64-bit ballots (one per voxel
//                  slot of a thread), always written, so the flags need no
//                  clearing.
//   k_interp_far   one thread per ballot word: for each flagged voxel, an
//                  exact outward search along z (stop once r^2 exceeds the
//                  best value: every candidate at offset r adds at least r^2),
//                  four offsets per round, then out and the distance word.
// Needed voxels far from B2 are few but their searches are long; keeping
// them out of the streaming waves keeps those waves short.  The distance word
// of every needed voxel goes to w2 (the adjoint reads it there).
struct ZsArgs {
    const uint32_t* w1;   // first-EDT words
    const uint32_t* gy;   // second EDT after its y pass
    uint32_t* w2;         // distance words at needed voxels
    const float* xq;      // may alias out
    float* out;
    uint64_t* flags;      // four ballot words per wave of k_interp_own
    int64_t nx, ny, nz;
    float eta_eb, power;
    bool blk;             // gy in the blocked layout [z][y/4][x][y%4] (else natural)
    const unsigned long long* b1count; // when set, the layout is chosen on the device (blocked_layout)
    const uint32_t* ovf;  // when set and raised, the y pass was redone by the banded pass (natural layout)
    const uint32_t* gx;   // k_interp_pre: the x-pass words of the second EDT (natural layout; w2 holds them)
    const unsigned long long* skip_sparse; // k_interp_far: when set, returns where sparse_b1 holds
};

// The y pass of the second EDT hands the needed-voxel search its words in the
// blocked layout where B1 covers at least 90% of the field (the first seed
// pass's estimate): needed voxels are then few, and the y pass's 16-byte
// stores pay.  Elsewhere many voxels are needed (up to two thirds of a
// field at rel. bound 1e-2) and the search's reads of natural rows touch a
// quarter of the cache lines, so the natural layout goes.  The y pass and
// the search read the same estimate and so agree on the layout.  The fused
// first-EDT search (k_edt1_yz) stands down below 80% on the same estimate.
__device__ __forceinline__ bool blocked_layout(const unsigned long long* b1count, uint64_t n)
{
    return *b1count * 10ull >= n * 9ull;
}

// index of voxel i's word in gy, and the distance between consecutive z-planes there
template <bool BLK>
__device__ __forceinline__ int64_t gy_index(const ZsArgs& a, int64_t i)
{
    if (!BLK)
        return i;
    const int64_t plane = a.nx * a.ny;
    const int64_t z = i / plane, r = i - z * plane;
    const int64_t y = r / a.nx, x = r - y * a.nx;
    return ((z * ((a.ny + 3) >> 2) + (y >> 2)) * a.nx + x) * 4 + (y & 3);
}
// the same in 32 bits (fields of fewer than 2^29 voxels); z of voxel i comes along
template <bool BLK>
__device__ __forceinline__ uint32_t gy_index32(const ZsArgs& a, uint32_t i, int& z)
{
    const uint32_t nx = (uint32_t)a.nx, plane = (uint32_t)(a.nx * a.ny);
    const uint32_t zz = i / plane, r = i - zz * plane;
    z = (int)zz;
    if (!BLK)
        return i;
    const uint32_t y = r / nx, x = r - y * nx;
    return ((zz * (uint32_t)((a.ny + 3) >> 2) + (y >> 2)) * nx + x) * 4u + (y & 3u);
}
template <bool BLK>
__device__ __forceinline__ int64_t gy_plane(const ZsArgs& a)
{
    return BLK ? ((a.ny + 3) >> 2) * 4 * a.nx : a.nx * a.ny;
}

// Loads of the y-pass words by 32-bit byte offset (buffer loads, fields below
// 2^30 voxels) or by 64-bit index.
template <bool BUF>
struct GyReader {
    const uint32_t* gy;
    __amdgpu_buffer_rsrc_t rs;
    __device__ __forceinline__ GyReader(const uint32_t* p, int64_t n)
        : gy(p), rs(__builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t*>(p), (short)0, BUF ? (int)(n * 4) : 0, 0x00020000))
    {
    }
    // word at voxel index i (byte offset o = 4 i when BUF)
    __device__ __forceinline__ uint32_t at(int64_t i) const
    {
        if (BUF)
            return __builtin_amdgcn_raw_buffer_load_b32(rs, (uint32_t)i * 4u, 0, 0);
        return gy[i];
    }
    // word at index i where take, else QAI_WORD_INF.  With buffer loads the
    // load is issued either way, at an offset past the buffer where it is not
    // wanted (the hardware returns 0 there without a memory access): no branch,
    // so several such loads stay in flight together.
    __device__ __forceinline__ uint32_t at_if(bool take, int64_t i) const
    {
        if (BUF) {
            const uint32_t v = __builtin_amdgcn_raw_buffer_load_b32(rs, take ? (uint32_t)i * 4u : 0xFFFFFFF0u, 0, 0);
            return take ? v : QAI_WORD_INF;
        }
        return take ? gy[i] : QAI_WORD_INF;
    }
};

// Exact d2 at voxel i (plane z) from the y-pass words: the outward search
// stops once r^2 exceeds the best value (every candidate at offset r adds at
// least r^2).  Each round issues all its loads before using any.  QAI_WORD_INF when the column holds no site.
template <bool BUF>
__device__ __forceinline__ uint32_t zsearch(const GyReader<BUF>& g, int64_t i, int64_t plane, int z, int nz)
{
    const uint32_t g0 = g.at(i);
    uint32_t best = (g0 == QAI_WORD_INF) ? QAI_WORD_INF : (g0 >> 2);
    auto round = [&](auto rc, int r0) {
        constexpr int R = decltype(rc)::value;
        uint32_t lo[R], hi[R];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int r = r0 + k;
            lo[k] = g.at_if(z - r >= 0, i - (int64_t)r * plane);
            hi[k] = g.at_if(z + r < nz, i + (int64_t)r * plane);
        }
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const uint32_t r2 = (uint32_t)((r0 + k) * (r0 + k));
            if (lo[k] != QAI_WORD_INF)
                best = min(best, (lo[k] >> 2) + r2);
            if (hi[k] != QAI_WORD_INF)
                best = min(best, (hi[k] >> 2) + r2);
        }
    };
    // offsets 1-4, 5-8, then 8 at a time
#pragma unroll 1
    for (int r0 = 1; r0 < nz;) {
        if ((best != QAI_WORD_INF && (uint32_t)(r0 * r0) > best) || (z - r0 < 0 && z + r0 >= nz))
            break;
        if (r0 < 9) {
            round(std::integral_constant<int, 4>(), r0);
            r0 += 4;
        } else if (r0 < 17) {
            round(std::integral_constant<int, 8>(), r0);
            r0 += 8;
        } else {
            round(std::integral_constant<int, 8>(), r0);
            r0 += 8;
        }
    }
    return best;
}

// out at a needed voxel from its distance value d2 (QAI_WORD_INF: no B2)
__device__ __forceinline__ float interp_val(const ZsArgs& a, uint32_t w1w, float xv, uint32_t d2)
{
    const bool none2 = d2 == QAI_WORD_INF;
    const float wt = idw_weight(word_d2(w1w), false, none2 ? 0u : d2, none2, a.power);
    return fmaf(wt, (float)word_sign(w1w) * a.eta_eb, xv);
}
// the same, with the distance word stored to w2
__device__ __forceinline__ float interp_at(const ZsArgs& a, int64_t i, uint32_t w1w, float xv, uint32_t d2)
{
    a.w2[i] = d2 == QAI_WORD_INF ? QAI_WORD_INF : (d2 << 2);
    return interp_val(a, w1w, xv, d2);
}

// step E where the weight does not need the search; false where it does (out
// then keeps x' for the second phase).  W2: store the distance word of a
// voxel on B2 (without it, w2 must already hold 0 there)
template <bool W2>
__device__ __forceinline__ bool interp_near(const ZsArgs& a, int64_t i, uint32_t w, float x, uint32_t g, float& o)
{
    const int s = word_sign(w);
    if (s == 0) {
        o = x;
    } else if (word_d2(w) == 0u) {
        o = fmaf(1.0f, (float)s * a.eta_eb, x); // on B1: w = 1
    } else if (g == 0u) {
        o = W2 ? interp_at(a, i, w, x, 0u) : interp_val(a, w, x, 0u); // on B2: w = 0
    } else {
        o = x;
        return false;
    }
    return true;
}

// PRE: the voxel's own word comes from the x pass (a.gx, natural layout)
// instead of the y pass.  A voxel lies on B2 exactly where its x-pass word is
// 0 (the voxel is itself a site), which is where the y-pass word is 0, so the
// flags and outputs are those of the y-pass form; the y pass may still be
// running.  The x-pass words hold 0 at B2 sites already, so w2 (the same
// buffer) is not written.
template <bool BUF, bool BLK, bool PRE = false>
__device__ __forceinline__ void interp_own(const ZsArgs& a)
{
    const int64_t n = a.nx * a.ny * a.nz;
    const GyReader<BUF> g(PRE ? a.gx : a.gy, PRE ? n : gy_plane<BLK>(a) * a.nz);
    const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    bool far[4] = {false, false, false, false};
    uint32_t w[4];
    float x[4], o[4];
    if (i0 + 4 <= n) {
        const uint4 wq = *reinterpret_cast<const uint4*>(a.w1 + i0);
        const float4 xq4 = *reinterpret_cast<const float4*>(a.xq + i0);
        w[0] = wq.x; w[1] = wq.y; w[2] = wq.z; w[3] = wq.w;
        x[0] = xq4.x; x[1] = xq4.y; x[2] = xq4.z; x[3] = xq4.w;
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            w[k] = i0 + k < n ? a.w1[i0 + k] : 0u; // beyond the field: S = 0, nothing done
            x[k] = i0 + k < n ? a.xq[i0 + k] : 0.0f;
        }
    }
    // the y-pass word of each needed voxel, the four loads in flight together
    uint32_t gv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const bool nd = word_sign(w[k]) != 0 && word_d2(w[k]) != 0u;
        int z;
        const int64_t j = PRE   ? min(i0 + k, n - 1)
                          : BUF ? (int64_t)gy_index32<BLK>(a, (uint32_t)min(i0 + k, n - 1), z)
                                : gy_index<BLK>(a, min(i0 + k, n - 1));
        gv[k] = g.at_if(nd, j);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
        far[k] = !interp_near<!PRE>(a, i0 + k, w[k], x[k], gv[k], o[k]);
    if (i0 + 4 <= n) {
        *reinterpret_cast<float4*>(a.out + i0) = make_float4(o[0], o[1], o[2], o[3]);
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (i0 + k < n)
                a.out[i0 + k] = o[k];
    }
    const uint64_t m0 = __ballot(far[0]), m1 = __ballot(far[1]), m2 = __ballot(far[2]), m3 = __ballot(far[3]);
    const int lane = threadIdx.x & 63;
    if (lane < 4) {
        const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
        a.flags[wave * 4 + lane] = lane == 0 ? m0 : (lane == 1 ? m1 : (lane == 2 ? m2 : m3));
    }
}

__device__ __forceinline__ bool zs_blocked(const ZsArgs& a)
{
    if (a.ovf && *a.ovf != 0u)
        return false;
    return a.b1count ? blocked_layout(a.b1count, (uint64_t)(a.nx * a.ny * a.nz)) : a.blk;
}

template <bool BUF>
__global__ __launch_bounds__(256) void k_interp_own(ZsArgs a)
{
    if (zs_blocked(a))
        interp_own<BUF, true>(a);
    else
        interp_own<BUF, false>(a);
}

// The same phase from the x-pass words, alongside the y pass (Plan1::aux).
template <bool BUF>
__global__ __launch_bounds__(256) void k_interp_pre(ZsArgs a)
{
    interp_own<BUF, false, true>(a);
}

// Which waves of k_interp_own a block of k_interp_far takes.  Searches of
// voxels in the same (y, x) column and nearby planes read the same y-pass
// lines, so where a plane holds whole waves (nx ny a multiple of 256) a block
// takes 8 consecutive waves (whole rows) of FAR_ZG = 4 consecutive planes (8
// planes: a few heavy blocks end the pass late; 2: the reuse falls off), and
// the blocks on each XCD (block b runs on XCD b % 8) walk a column group
// through a chunk of 64 planes in order: the lines they read stay in that
// XCD's L2.
// Chunk c of column group j goes to XCD (j + c) % 8, so every XCD takes
// planes from the whole depth (the density of far voxels follows that of B2,
// plane by plane); column groups are taken from both y faces inward, where B2
// never lies and every needed voxel is flagged, so those heavy rows come
// first.  Otherwise a block takes 64 waves spaced gridDim.x apart.
struct FarMap {
    int64_t wpp;      // waves per plane (0: the spaced mapping)
    int64_t pb, zb;   // 8-wave groups per plane, FAR_ZG-plane groups
    int64_t ncx;      // chunks of FAR_ZC plane groups per XCD and column group
};
constexpr int FAR_ZG = 4, FAR_ZC = 64 / FAR_ZG;

__device__ __forceinline__ int64_t far_wave(const FarMap& f, int64_t nz, int64_t nwaves, int lw)
{
    if (f.wpp == 0) {
        const int64_t w = (int64_t)blockIdx.x + (int64_t)lw * gridDim.x;
        return w < nwaves ? w : -1;
    }
    const int k = blockIdx.x & 7;
    const int64_t u = blockIdx.x >> 3;
    const int64_t unit = u / FAR_ZC, j = unit / f.ncx;
    const int64_t zc = ((k - j) % 8 + 8) % 8 + 8 * (unit % f.ncx);
    const int64_t zb = zc * FAR_ZC + u % FAR_ZC;
    if (j >= f.pb || zb >= f.zb)
        return -1;
    if ((lw >> 3) >= FAR_ZG)
        return -1;
    const int64_t cg = (j & 1) ? f.pb - 1 - (j >> 1) : (j >> 1);
    const int64_t z = zb * FAR_ZG + (lw >> 3), p = cg * 8 + (lw & 7);
    return (z < nz && p < f.wpp) ? z * f.wpp + p : -1;
}

// A block takes the four flag words of up to 64 waves of k_interp_own (far_wave).
// The block's flagged voxels are listed in LDS (block-wide prefix sum of the
// word popcounts) and dealt one per thread; lists longer than the LDS window
// go in several rounds.
constexpr int FAR_LIST = 1024;

template <bool BUF>
__global__ __launch_bounds__(256) void k_interp_far(ZsArgs a, int64_t nwords, FarMap fm)
{
    constexpr int L = FAR_LIST;
    __shared__ int64_t list[L];
    __shared__ int wsum[4];
    if (a.skip_sparse && sparse_b1(a.skip_sparse, (uint64_t)(a.nx * a.ny * a.nz)))
        return; // the whole z pass runs instead
    const bool blk = zs_blocked(a);
    const int64_t plane = a.nx * a.ny, gplane = blk ? gy_plane<true>(a) : gy_plane<false>(a);
    const GyReader<BUF> g(a.gy, gplane * a.nz);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t grp = far_wave(fm, a.nz, nwords / 4, tid >> 2); // wave of k_interp_own
    const int64_t wi = grp * 4 + (tid & 3);
    const uint64_t m = grp >= 0 ? a.flags[wi] : 0ull;
    const int c = __popcll(m);
    // exclusive prefix of c over the block
    int incl = c;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int v = __shfl_up(incl, d);
        if (lane >= d)
            incl += v;
    }
    if (lane == 63)
        wsum[wv] = incl;
    lds_barrier();
    int before = 0, total = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        before += k < wv ? wsum[k] : 0;
        total += wsum[k];
    }
    const int off = before + incl - c;
    const int64_t base = (wi >> 2) * 256 + (wi & 3); // voxel of bit l: base + 4 l
#pragma unroll 1
    for (int w0 = 0; w0 < total; w0 += L) {
        // this thread's flagged voxels that fall in list window [w0, w0 + L)
        if (off < w0 + L && off + c > w0) {
            uint64_t mm = m;
            int p = off;
            while (mm) {
                const int l = __ffsll((unsigned long long)mm) - 1;
                mm &= mm - 1ull;
                if (p >= w0 && p < w0 + L)
                    list[p - w0] = base + 4 * (int64_t)l;
                ++p;
            }
        }
        lds_barrier();
        const int cnt = min(L, total - w0);
#pragma unroll 1
        for (int j = tid; j < cnt; j += 256) {
            const int64_t i = list[j];
            const uint32_t w = a.w1[i];
            const float xv = a.xq[i];
            int z;
            const int64_t jg = BUF ? (int64_t)(blk ? gy_index32<true>(a, (uint32_t)i, z) : gy_index32<false>(a, (uint32_t)i, z))
                                   : (blk ? gy_index<true>(a, i) : gy_index<false>(a, i));
            if (!BUF)
                z = (int)(i / plane);
            const uint32_t d2 = zsearch<BUF>(g, jg, gplane, z, (int)a.nz);
            a.out[i] = interp_at(a, i, w, xv, d2);
        }
        if (w0 + L < total) // after the last window, threads without searches leave at once
            lds_barrier();
    }
}

// Step E over a 2-D field with the second EDT's y pass done only where the
// weight needs it (S != 0 off B1): at such a voxel the outward search of
// k_env_direct over the x-pass words (a.gx), same order and stop rule; every
// other voxel is finished as interp_near finishes it.  One thread per voxel,
// 256 consecutive voxels of a row per workgroup: a wave's searches read
// consecutive words of the same rows.  The distance word of a needed voxel
// goes to w2 (a buffer apart from a.gx, which other searches still read).
__global__ __launch_bounds__(256) void k_interp_dir(ZsArgs a)
{
    const int64_t n = a.ny, stride = a.nx;
    const int64_t nxb = (a.nx + 255) >> 8;
    const uint64_t units = (uint64_t)(a.ny * nxb);
    for (uint64_t u = blockIdx.x; u < units; u += gridDim.x) {
        const int64_t p = (int64_t)(u / (uint64_t)nxb), xb = (int64_t)(u % (uint64_t)nxb);
        const int64_t x = xb * 256 + threadIdx.x;
        if (x >= a.nx)
            continue;
        const int64_t i = p * a.nx + x;
        const uint32_t w = a.w1[i];
        const float xv = a.xq[i];
        const int s = word_sign(w);
        if (s == 0 || word_d2(w) == 0u) {
            a.out[i] = s == 0 ? xv : fmaf(1.0f, (float)s * a.eta_eb, xv); // S = 0, or on B1 (w = 1)
            continue;
        }
        uint32_t best = a.gx[i];
        bool done = false;
        for (int64_t d0 = 1; d0 < n && !done; d0 += 4) {
            uint32_t lo[4], hi[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int64_t d = d0 + k;
                lo[k] = (p - d >= 0) ? a.gx[i - d * stride] : QAI_WORD_INF;
                hi[k] = (p + d < n) ? a.gx[i + d * stride] : QAI_WORD_INF;
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int64_t d = d0 + k;
                const uint32_t d2s = (uint32_t)d * (uint32_t)d << 2;
                if (done || d >= n || d2s > (best | 3u) || (p - d < 0 && p + d >= n)) {
                    done = true;
                    continue;
                }
                if (p - d >= 0) {
                    const uint32_t cand = word_add(lo[k], d2s);
                    if ((cand >> 2) <= (best >> 2))
                        best = cand;
                }
                if (p + d < n) {
                    const uint32_t cand = word_add(hi[k], d2s);
                    if ((cand >> 2) < (best >> 2))
                        best = cand;
                }
            }
        }
        a.out[i] = interp_at(a, i, w, xv, best == QAI_WORD_INF ? QAI_WORD_INF : (best >> 2));
    }
}

// Geometry of the two phases: a thread of the streaming phase takes four
// voxels; buffer loads by 32-bit byte offset while gy (natural or blocked)
// stays below 2^31 bytes.
static hipError_t interp_geom(const ZsArgs& a, bool force_wide, int64_t& blocks, bool& buf)
{
    const int64_t n = a.nx * a.ny * a.nz;
    if ((((uintptr_t)a.w1 | (uintptr_t)a.xq | (uintptr_t)a.out) & 15u) != 0)
        return hipErrorInvalidValue; // the caller takes the unfused path instead
    blocks = (n + 1023) / 1024;
    if (blocks > 0x7FFFFFFF)
        return hipErrorInvalidValue;
    buf = word_capacity(a.nz, a.ny, a.nx) < ((int64_t)1 << 29) && !force_wide;
    return hipSuccess;
}

// the streaming phase: from the y-pass words (k_interp_own) or, pre, from the
// x-pass words (k_interp_pre)
static hipError_t launch_interp_stream(const ZsArgs& a, bool force_wide, bool pre, hipStream_t s)
{
    int64_t blocks;
    bool buf;
    QAI_TRY(interp_geom(a, force_wide, blocks, buf));
    const dim3 grid((unsigned)blocks), blk(256);
    if (pre)
        return buf ? launch_checked(k_interp_pre<true>, grid, blk, 0, s, a)
                   : launch_checked(k_interp_pre<false>, grid, blk, 0, s, a);
    return buf ? launch_checked(k_interp_own<true>, grid, blk, 0, s, a)
               : launch_checked(k_interp_own<false>, grid, blk, 0, s, a);
}

template <bool BUF>
static hipError_t launch_interp_far_t(const ZsArgs& a, int64_t blocks, hipStream_t s)
{
    const int64_t nwords = blocks * 16; // flag_bytes(n) / 8
    const int64_t plane = a.nx * a.ny;
    FarMap fm{0, 0, 0, 0};
    int64_t grid = (nwords / 4 + 63) / 64;
    if (plane % 256 == 0) {
        fm.wpp = plane / 256;
        fm.pb = (fm.wpp + 7) / 8;
        fm.zb = (a.nz + FAR_ZG - 1) / FAR_ZG;
        fm.ncx = ((fm.zb + FAR_ZC - 1) / FAR_ZC + 7) / 8;
        grid = 8 * fm.pb * fm.ncx * FAR_ZC;
    }
    return launch_checked(k_interp_far<BUF>, dim3((unsigned)grid), dim3(256), 0, s, a, nwords, fm);
}

// the search phase over the voxels the streaming phase flagged
static hipError_t launch_interp_far(const ZsArgs& a, bool force_wide, hipStream_t s)
{
    int64_t blocks;
    bool buf;
    QAI_TRY(interp_geom(a, force_wide, blocks, buf));
    return buf ? launch_interp_far_t<true>(a, blocks, s) : launch_interp_far_t<false>(a, blocks, s);
}

static uint32_t grid_cap(uint64_t units, uint64_t cap);

static hipError_t launch_interp_dir(const ZsArgs& a, hipStream_t s)
{
    const uint64_t units = (uint64_t)(a.ny * ((a.nx + 255) >> 8));
    return launch_checked(k_interp_dir, dim3(grid_cap(units, 1u << 20)), dim3(256), 0, s, a);
}

// --------------------------------------------------------- envelope pass
// Exact 1-D minimisation D(i) = min_j g(j) + (i - j)^2 along the pass axis
// for a tile of adjacent x-columns, whole lines staged in LDS.  Candidates
// are visited outward from i (offset d = 1, 2, ...); the search stops once
// d^2 exceeds the best value found, since every farther candidate is at
// least d^2.  At equal value the lower coordinate wins (left candidates win
// ties, right ones need to be strictly better), the choice Algorithm 1's
// strict comparisons make.
template <int AXIS>
__global__ __launch_bounds__(1024) void k_env_window(EnvArgs a)
{
    extern __shared__ __align__(16) uint32_t tile[];
    const int txl = a.tx_log2;
    const int Tx = 1 << txl;
    const int64_t n = (AXIS == 1) ? a.ny : a.nz;
    const int64_t stride = (AXIS == 1) ? a.nx : a.nx * a.ny;
    const int64_t nxb = (a.nx + Tx - 1) >> txl;
    const int total = (int)(n << txl);
    if (a.gate && *a.gate == 0u)
        return; // gated pass not needed (uniform over the grid)

    for (uint64_t t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
        const uint64_t tl = xcd_remap(t, a.ntiles);
        const int64_t xb = (int64_t)(tl % (uint64_t)nxb), o = (int64_t)(tl / (uint64_t)nxb);
        const int64_t x0 = xb << txl;
        const int64_t base = (AXIS == 1) ? o * a.nx * a.ny + x0 : o * a.nx + x0;
        __syncthreads();
        int any = 0;
        for (int i = threadIdx.x; i < total; i += blockDim.x) {
            const int r = i >> txl, c = i & (Tx - 1);
            const uint32_t v = (x0 + c < a.nx) ? a.win[base + (int64_t)r * stride + c] : QAI_WORD_INF;
            tile[i] = v;
            any |= (v != QAI_WORD_INF);
        }
        // a tile without any site (e.g. the domain's edge planes in the first EDT)
        // keeps every voxel at "no site": skip the searches
        const bool live = __syncthreads_or(any) != 0;
        for (int i = threadIdx.x; i < total; i += blockDim.x) {
            const int r = i >> txl, c = i & (Tx - 1);
            if (x0 + c >= a.nx)
                continue;
            uint32_t best = tile[i];
            for (int d = 1; live && d < n; ++d) {
                const uint32_t d2s = (uint32_t)d * (uint32_t)d << 2;
                if (d2s > (best | 3u))
                    break;
                const int lo = r - d, hi = r + d;
                if (lo < 0 && hi >= n)
                    break;
                if (lo >= 0) {
                    const uint32_t cand = word_add(tile[(lo << txl) + c], d2s);
                    if ((cand >> 2) <= (best >> 2))
                        best = cand;
                }
                if (hi < n) {
                    const uint32_t cand = word_add(tile[(hi << txl) + c], d2s);
                    if ((cand >> 2) < (best >> 2))
                        best = cand;
                }
            }
            a.w[base + (int64_t)r * stride + c] = best;
        }
    }
}

// Direct outward search for short owner distances: one thread per voxel,
// 256 consecutive voxels of one x-line per workgroup, the candidates read
// straight from the pass input (the lines a voxel's search reads are the
// neighbouring workgroups' own lines, so the caches serve most of them).
// Every voxel of the field works at once, whatever the number of column
// tiles: the choice for passes whose tiles are too few to fill the GPU.  Same
// order and tie rule as k_env_window; four offsets per round with all eight
// loads in flight.
template <int AXIS>
__global__ __launch_bounds__(256) void k_env_direct(EnvArgs a)
{
    if (a.gate && *a.gate == 0u)
        return; // gated pass not needed (uniform over the grid)
    const int64_t n = (AXIS == 1) ? a.ny : a.nz;
    const int64_t stride = (AXIS == 1) ? a.nx : a.nx * a.ny;
    const int64_t nxb = (a.nx + 255) >> 8;
    const uint64_t units = (uint64_t)(a.nz * a.ny * nxb);
    for (uint64_t u = blockIdx.x; u < units; u += gridDim.x) {
        const int64_t line = (int64_t)(u / (uint64_t)nxb), xb = (int64_t)(u % (uint64_t)nxb);
        const int64_t x = xb * 256 + threadIdx.x;
        if (x >= a.nx)
            continue;
        const int64_t p = (AXIS == 1) ? line % a.ny : line / a.ny; // position along the pass axis
        const int64_t i = line * a.nx + x;
        uint32_t best = a.win[i];
        bool done = false;
        for (int64_t d0 = 1; d0 < n && !done; d0 += 4) {
            uint32_t lo[4], hi[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int64_t d = d0 + k;
                lo[k] = (p - d >= 0) ? a.win[i - d * stride] : QAI_WORD_INF;
                hi[k] = (p + d < n) ? a.win[i + d * stride] : QAI_WORD_INF;
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int64_t d = d0 + k;
                const uint32_t d2s = (uint32_t)d * (uint32_t)d << 2;
                if (done || d >= n || d2s > (best | 3u) || (p - d < 0 && p + d >= n)) {
                    done = true;
                    continue;
                }
                if (p - d >= 0) {
                    const uint32_t cand = word_add(lo[k], d2s);
                    if ((cand >> 2) <= (best >> 2))
                        best = cand;
                }
                if (p + d < n) {
                    const uint32_t cand = word_add(hi[k], d2s);
                    if ((cand >> 2) < (best >> 2))
                        best = cand;
                }
            }
        }
        a.w[i] = best;
    }
}

// Streaming outward search for short owner distances (the first EDT, whose
// sites are dense): one lane per column, 64 adjacent columns per wave, the
// column read once in blocks of 8 rows into a per-wave ring of 32 rows in LDS.
// A row is settled from the ring when its outward search (same order and tie
// rule as k_env_window) ends within H rows; rows with no site within H rows
// are settled after the sweep by the same search over the whole column, and a
// column without any site stays at "no site".
template <int AXIS, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_env_swin(EnvArgs a)
{
    constexpr int H = 8, RN = 32;
    __shared__ uint32_t ring[WPB * RN * 64];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    uint32_t* const rl = ring + wv * RN * 64 + lane;
    const int n = (int)((AXIS == 1) ? a.ny : a.nz);
    const int64_t stride = (AXIS == 1) ? a.nx : a.nx * a.ny;
    const int64_t nxb = (a.nx + 63) >> 6;
    const uint64_t ngroups = (a.ntiles + WPB - 1) / WPB;
    if (a.gate && *a.gate == 0u)
        return; // gated pass not needed (uniform over the grid)

    // tiles in dispatch order (as in k_env_lane2: no shared lines, work that
    // follows the density of sites plane by plane)
    for (uint64_t t = blockIdx.x; t < ngroups; t += gridDim.x) {
        const uint64_t tile = t * WPB + wv;
        if (tile >= a.ntiles)
            continue;
        const int64_t xb = (int64_t)(tile % (uint64_t)nxb), o = (int64_t)(tile / (uint64_t)nxb);
        const int64_t x0 = xb * 64;
        const bool valid = x0 + lane < a.nx;
        const int64_t tb = ((AXIS == 1) ? o * a.nx * a.ny : o * a.nx) + x0;
        const uint32_t* __restrict__ inb = a.win + tb;
        uint32_t* const outb = a.w + tb;
        const uint32_t us = (uint32_t)stride;
        const uint32_t uc = valid ? (uint32_t)lane : 0u;
        const int nb = (n + 7) >> 3;
        int pf = 0x7fffffff, pl = -1; // first and last row left unresolved by the ring search
        bool seen = false;            // any site in the column
        uint32_t sm = 0u;             // bit (row & 31): that ring row holds a site

        auto finalize = [&](int f) {
            uint32_t best = rl[(f & (RN - 1)) * 64];
            // no site within +-H rows: unresolved without searching
            const bool near = (__builtin_rotateright32(sm, (uint32_t)(f - H) & 31u) & ((2u << (2 * H)) - 1u)) != 0u;
            if ((best >> 2) != 0u && !near) {
                pf = min(pf, f);
                pl = f;
            } else if ((best >> 2) != 0u) {
                int d = 1;
                for (; d <= H; ++d) {
                    const uint32_t d2s = (uint32_t)d * (uint32_t)d << 2;
                    if (d2s > (best | 3u))
                        break;
                    const int lo = f - d, hi = f + d;
                    if (lo < 0 && hi >= n)
                        break;
                    if (lo >= 0) {
                        const uint32_t cand = word_add(rl[(lo & (RN - 1)) * 64], d2s);
                        if ((cand >> 2) <= (best >> 2))
                            best = cand;
                    }
                    if (hi < n) {
                        const uint32_t cand = word_add(rl[(hi & (RN - 1)) * 64], d2s);
                        if ((cand >> 2) < (best >> 2))
                            best = cand;
                    }
                }
                if (d > H) {
                    // unresolved inside the ring: settled after the sweep
                    pf = min(pf, f);
                    pl = f;
                }
            }
            // spare lanes of a partial tile read column x0 and store lane 0's value there
            outb[(uint32_t)f * us + uc] = best;
        };

        uint32_t A[8], B[8];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            A[k] = inb[(uint32_t)min(k, n - 1) * us + uc];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            B[k] = inb[(uint32_t)min(8 + k, n - 1) * us + uc];
        // block b: store rows 8b..8b+7 into the ring, prefetch block b+2, finalize
        // block b-1 (its searches reach 8 rows into block b).  Pairs of blocks
        // without guards (a guarded use of a prefetched block made the compiler
        // wait for every outstanding load at the loop's back edge), then an odd
        // last block.
        auto ring_put = [&](int b, const uint32_t (&R)[8]) {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                rl[(((b * 8) + k) & (RN - 1)) * 64] = R[k];
                seen |= R[k] != QAI_WORD_INF;
                sm = (R[k] != QAI_WORD_INF) ? (sm | (1u << (((b * 8) + k) & 31))) : (sm & ~(1u << (((b * 8) + k) & 31)));
            }
        };
        int b = 0;
        for (; b + 2 <= nb; b += 2) {
            ring_put(b, A);
#pragma unroll
            for (int k = 0; k < 8; ++k)
                A[k] = inb[(uint32_t)min((b + 2) * 8 + k, n - 1) * us + uc];
            if (b >= 1) {
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    finalize((b - 1) * 8 + k);
            }
            ring_put(b + 1, B);
#pragma unroll
            for (int k = 0; k < 8; ++k)
                B[k] = inb[(uint32_t)min((b + 3) * 8 + k, n - 1) * us + uc];
#pragma unroll
            for (int k = 0; k < 8; ++k)
                finalize(b * 8 + k);
        }
        if (b < nb) {
            ring_put(b, A);
            if (b >= 1) {
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    finalize((b - 1) * 8 + k);
            }
        }
        // the last block
        for (int f = (nb - 1) * 8; f < n; ++f)
            finalize(f);
        // rows farther than H from every useful site: exact outward search over
        // the whole column (a column without any site stays at "no site")
        if (__ballot(seen && pl >= 0 && valid)) {
            if (seen && pl >= 0 && valid) {
                for (int f = pf; f <= pl; ++f) {
                    uint32_t best = outb[(uint32_t)f * us + uc];
                    if (best != QAI_WORD_INF && (best >> 2) < (uint32_t)((H + 1) * (H + 1)))
                        continue;
                    best = inb[(uint32_t)f * us + uc];
                    for (int d = 1; d < n; ++d) {
                        const uint32_t d2s = (uint32_t)d * (uint32_t)d << 2;
                        if (d2s > (best | 3u))
                            break;
                        const int lo = f - d, hi = f + d;
                        if (lo < 0 && hi >= n)
                            break;
                        if (lo >= 0) {
                            const uint32_t cand = word_add(inb[(uint32_t)lo * us + uc], d2s);
                            if ((cand >> 2) <= (best >> 2))
                                best = cand;
                        }
                        if (hi < n) {
                            const uint32_t cand = word_add(inb[(uint32_t)hi * us + uc], d2s);
                            if ((cand >> 2) < (best >> 2))
                                best = cand;
                        }
                    }
                    outb[(uint32_t)f * us + uc] = best;
                }
            }
        }
    }
}

// RemoveEDT(g_u, g_v, g_w, u, v) with sites u < v < w (Section III-B): true
// when v's cell between u and w is empty.  Products reach 2^44: int64.
__device__ __forceinline__ bool remove_mid(uint32_t gu, uint32_t gv, uint32_t gw, int u, int v, int w)
{
    const int64_t a = v - u, b = w - v, c = w - u;
    return c * (int64_t)gv - b * (int64_t)gu - a * (int64_t)gw - a * b * c > 0;
}

__device__ __forceinline__ uint32_t fval(uint32_t g, int s, int p)
{
    const int d = p - s;
    return g + (uint32_t)(d * d);
}

// Wave-per-column variant of the banded envelope.  The B bands of a column
// are B consecutive lanes of one wavefront (B a power of two <= 64), so the
// pairwise merges, the survivor masks and the search for a starting site are
// wave-local (shuffles, ballots, a wave-scope fence) and a tile needs only
// three workgroup barriers.  LDS holds each column as B bands of M words plus
// one pad word (band-parallel accesses hit distinct banks); results are
// collected in registers, written back over the tile and stored coalesced.
template <int M>
struct Band2 {
    int colstride; // words per column: B * (M + 1) + 1 (odd)
    uint32_t* G;
    int16_t* PREV;
    int16_t* NEXT;
    __device__ __forceinline__ int at(int c, int p) const
    {
        return c * colstride + (p / M) * (M + 1) + (p % M);
    }
};

template <int AXIS, int M>
__global__ __launch_bounds__(1024) void k_env_band2(EnvArgs a, int lb)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int B = 1 << lb;
    const int txl = a.tx_log2;
    const int Tx = 1 << txl;
    const int n = (int)((AXIS == 1) ? a.ny : a.nz);
    const int64_t stride = (AXIS == 1) ? a.nx : a.nx * a.ny;
    const int64_t nxb = (a.nx + Tx - 1) >> txl;
    Band2<M> L;
    L.colstride = B * (M + 1) + 1;
    L.G = (uint32_t*)smem;
    L.PREV = (int16_t*)(L.G + (size_t)L.colstride * Tx);
    L.NEXT = L.PREV + (size_t)L.colstride * Tx;

    if (a.gate && *a.gate == 0u)
        return; // gated pass not needed (uniform over the grid)
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int b = lane & (B - 1);                      // band of this lane
    const int seg = lane & ~(B - 1);                   // first lane of this column's bands
    const int c = ((tid >> 6) << (6 - lb)) + (lane >> lb); // column in the tile
    const int p0 = b * M;
    const int cbase = c * L.colstride + b * (M + 1);   // LDS index of position p0
    const int total = n << txl;

    for (uint64_t t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
        const uint64_t tl = xcd_remap(t, a.ntiles);
        const int64_t xb = (int64_t)(tl % (uint64_t)nxb), o = (int64_t)(tl / (uint64_t)nxb);
        const int64_t x0 = xb << txl;
        const int64_t base = (AXIS == 1) ? o * a.nx * a.ny + x0 : o * a.nx + x0;
        __syncthreads();
        for (int i = tid; i < total; i += blockDim.x) {
            const int r = i >> txl, cc = i & (Tx - 1);
            L.G[L.at(cc, r)] = (x0 + cc < a.nx) ? a.win[base + (int64_t)r * stride + cc] : QAI_WORD_INF;
        }
        for (int i = tid; i < ((B * M - n) << txl); i += blockDim.x) // padding positions n .. B*M-1
            L.G[L.at(i & (Tx - 1), n + (i >> txl))] = QAI_WORD_INF;
        __syncthreads();

        // 1. envelope of each band (Algorithm 1's stack as a linked list)
        int head = -1, top = -1;
        {
            int second = -1;
            uint32_t gtop = 0, gsec = 0;
#pragma unroll 4
            for (int j = 0; j < M; ++j) {
                const int p = p0 + j;
                const uint32_t w = L.G[cbase + j];
                if (w == QAI_WORD_INF)
                    continue;
                const uint32_t g = w >> 2;
                for (int it = 0; it < M && second >= 0 && remove_mid(gsec, gtop, g, second, top, p); ++it) {
                    L.PREV[L.at(c, top)] = -2;
                    top = second;
                    gtop = gsec;
                    second = L.PREV[L.at(c, second)];
                    gsec = second >= 0 ? (L.G[L.at(c, second)] >> 2) : 0u;
                }
                L.PREV[cbase + j] = (int16_t)top;
                if (top >= 0)
                    L.NEXT[L.at(c, top)] = (int16_t)p;
                else
                    head = p;
                second = top;
                gsec = gtop;
                top = p;
                gtop = g;
            }
            if (top >= 0)
                L.NEXT[L.at(c, top)] = -1;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        // 2. wave-local pairwise merges; (head, top) describe this lane's super-band
        for (int span = 1; span < B; span <<= 1) {
            const int src = seg + ((b + span) & (B - 1));
            const int rh = __shfl(head, src);
            const int rt = __shfl(top, src);
            if ((b & (2 * span - 1)) == 0 && b + span < B) {
                if (top < 0) {
                    head = rh;
                    top = rt;
                } else if (rt >= 0) {
                    int t1 = top, t0 = L.PREV[L.at(c, t1)];
                    int h1 = rh, h2 = L.NEXT[L.at(c, h1)];
                    uint32_t g_t1 = L.G[L.at(c, t1)] >> 2, g_h1 = L.G[L.at(c, h1)] >> 2;
                    uint32_t g_t0 = t0 >= 0 ? (L.G[L.at(c, t0)] >> 2) : 0u;
                    uint32_t g_h2 = h2 >= 0 ? (L.G[L.at(c, h2)] >> 2) : 0u;
                    for (int it = 0; it < n; ++it) {
                        if (t0 >= 0 && remove_mid(g_t0, g_t1, g_h1, t0, t1, h1)) {
                            L.PREV[L.at(c, t1)] = -2;
                            t1 = t0;
                            g_t1 = g_t0;
                            t0 = L.PREV[L.at(c, t0)];
                            g_t0 = t0 >= 0 ? (L.G[L.at(c, t0)] >> 2) : 0u;
                            continue;
                        }
                        if (h2 >= 0 && remove_mid(g_t1, g_h1, g_h2, t1, h1, h2)) {
                            L.PREV[L.at(c, h1)] = -2;
                            h1 = h2;
                            g_h1 = g_h2;
                            h2 = L.NEXT[L.at(c, h2)];
                            g_h2 = h2 >= 0 ? (L.G[L.at(c, h2)] >> 2) : 0u;
                            continue;
                        }
                        break;
                    }
                    L.NEXT[L.at(c, t1)] = (int16_t)h1;
                    L.PREV[L.at(c, h1)] = (int16_t)t1;
                    top = rt;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }

        // survivors of this band, and the column's survivor mask
        int first = -1, last = -1;
        for (int j = 0; j < M; ++j) {
            if (L.G[cbase + j] != QAI_WORD_INF && L.PREV[cbase + j] != -2) {
                if (first < 0)
                    first = p0 + j;
                last = p0 + j;
            }
        }
        const uint64_t ball = __ballot(first >= 0);
        const uint64_t mk = (B == 64) ? ball : ((ball >> seg) & ((1ull << B) - 1ull));
        int s = first;
        {
            const uint64_t below = mk & ((1ull << b) - 1ull);
            const int lsrc = below ? seg + 63 - __clzll(below) : lane;
            const int fsrc = mk ? seg + __ffsll((unsigned long long)mk) - 1 : lane;
            const int lastv = __shfl(last, lsrc);
            const int firstv = __shfl(first, fsrc);
            if (s < 0)
                s = below ? lastv : (mk ? firstv : -1);
        }

        // 3. query: owner of p0 by a unimodal walk, then monotone advance
        uint32_t res[M];
        if (s < 0) {
#pragma unroll
            for (int j = 0; j < M; ++j)
                res[j] = QAI_WORD_INF;
        } else {
            int o = s;
            uint32_t wo = L.G[L.at(c, o)];
            for (int it = 0; it < n; ++it) {
                const int pv = L.PREV[L.at(c, o)];
                if (pv < 0)
                    break;
                const uint32_t wp = L.G[L.at(c, pv)];
                if (fval(wp >> 2, pv, p0) > fval(wo >> 2, o, p0))
                    break;
                o = pv;
                wo = wp;
            }
            int nx_ = L.NEXT[L.at(c, o)];
            uint32_t wn = nx_ >= 0 ? L.G[L.at(c, nx_)] : 0u;
#pragma unroll
            for (int j = 0; j < M; ++j) {
                const int p = p0 + j;
                for (int it = 0; it < n && nx_ >= 0 && fval(wn >> 2, nx_, p) < fval(wo >> 2, o, p); ++it) {
                    o = nx_;
                    wo = wn;
                    nx_ = L.NEXT[L.at(c, o)];
                    wn = nx_ >= 0 ? L.G[L.at(c, nx_)] : 0u;
                }
                const int d = p - o;
                res[j] = wo + ((uint32_t)(d * d) << 2);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int j = 0; j < M; ++j)
            L.G[cbase + j] = res[j];
        __syncthreads();

        // coalesced store
        for (int i = tid; i < total; i += blockDim.x) {
            const int r = i >> txl, cc = i & (Tx - 1);
            if (x0 + cc >= a.nx)
                continue;
            a.w[base + (int64_t)r * stride + cc] = L.G[L.at(cc, r)];
        }
    }
}

// RemoveEDT in 32 bits with full-rate 24-bit multiplies: exact when the line
// length n < 2^12 and every site value g < 2^24 satisfy n g + n^3 / 4 < 2^31
// (with a + b = c <= n the positive term c g_v is below n g and the negative
// ones sum below n g + n^3 / 4).  The launcher checks this from the extents.
__device__ __forceinline__ bool remove_mid24(uint32_t gu, uint32_t gv, uint32_t gw, int u, int v, int w)
{
    const uint32_t a = (uint32_t)(v - u), b = (uint32_t)(w - v), c = (uint32_t)(w - u);
    const int32_t t = (int32_t)__umul24(c, gv) - (int32_t)__umul24(b, gu) - (int32_t)__umul24(a, gw) -
                      (int32_t)__umul24(__umul24(a, b), c);
    return t > 0;
}

template <bool SMALL>
__device__ __forceinline__ bool remove_sel(uint32_t gu, uint32_t gv, uint32_t gw, int u, int v, int w)
{
    if (SMALL)
        return remove_mid24(gu, gv, gw, u, v, w);
    return remove_mid(gu, gv, gw, u, v, w);
}

__device__ __forceinline__ uint32_t sq24(int d) { return (uint32_t)__mul24(d, d); }

// Streaming exact lower envelope: one lane per column, 64 adjacent x-columns
// per wavefront, one sweep along the line (Algorithm 1 made online).
//
// At row i the lane pushes site i on Algorithm 1's stack (popping with
// RemoveEDT), then emits every row e whose answer can no longer change: a
// future site j > i contributes at least (j - e)^2 >= (i+1-e)^2, so e is
// final once its best value is <= (i+1-e)^2 (a future site of equal value
// has the higher coordinate and loses the tie).  A finalised owner cannot be
// removed later (it would have to be strictly dominated at e), so everything
// below the query pointer is dropped and only the live window
// [owner(e), top] is kept, in an LDS ring of C entries per lane.  Emission is
// synchronised per group of 16 lanes, so stores are 64-byte row segments
// while the live window only has to cover the group's slowest column.  A
// column whose window outgrows the ring is finished afterwards by the whole
// wave with an exact outward search over the untouched input column (same
// result, different cost).
template <int AXIS, int C, bool SMALL>
__global__ __launch_bounds__(128) void k_env_stream(EnvArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int nwv = blockDim.x >> 6;
    uint32_t* rw = (uint32_t*)smem + (size_t)wv * C * 64;
    uint16_t* rh = (uint16_t*)((uint32_t*)smem + (size_t)nwv * C * 64) + (size_t)wv * C * 64;
    const int n = (int)((AXIS == 1) ? a.ny : a.nz);
    const int64_t stride = (AXIS == 1) ? a.nx : a.nx * a.ny;
    const int64_t nxb = (a.nx + 63) >> 6;
    const uint64_t ngroups = (a.ntiles + nwv - 1) / nwv;
    const int grp = lane >> 4;
    const uint64_t gmask = 0xFFFFull << (grp * 16);

    for (uint64_t t = blockIdx.x; t < ngroups; t += gridDim.x) {
        const uint64_t tile = (uint64_t)__builtin_amdgcn_readfirstlane((int)(xcd_remap(t, ngroups) * nwv + wv));
        if (tile >= a.ntiles)
            continue;
        const int64_t xb = (int64_t)(tile % (uint64_t)nxb), o = (int64_t)(tile / (uint64_t)nxb);
        const int64_t x0 = xb * 64;
        const bool valid = x0 + lane < a.nx;
        const int col = valid ? lane : 0; // invalid lanes read a valid word and ignore it
        const int64_t tb = ((AXIS == 1) ? o * a.nx * a.ny : o * a.nx) + x0;
        const uint32_t* __restrict__ inp = a.win + tb;
        uint32_t* __restrict__ outp = a.w + tb;

        // live window [lo, top] of Algorithm 1's stack in the ring (logical
        // indices; slot = index mod C); only these scalars cross rows
        int lo = 0, top = -1;
        bool ovf = !valid;
        int e = 0;                       // next row to emit (uniform within the lane's group)
        uint32_t bestB = QAI_WORD_INF;   // value at row e over the sites seen so far
        uint32_t bestW = QAI_WORD_INF;   // the corresponding word (value and sign code)
        uint32_t* const rwl = rw + lane;
        uint16_t* const rhl = rh + lane;
#define RW(k) rwl[((k) & (C - 1)) * 64]
#define RH(k) ((int)rhl[((k) & (C - 1)) * 64])

        // owner of row r among the live entries (the pointer only moves forward)
        auto refresh = [&](int r) {
            if (top < lo) {
                bestB = QAI_WORD_INF;
                bestW = QAI_WORD_INF;
                return;
            }
            uint32_t wl = RW(lo);
            int hl = RH(lo);
            uint32_t bl = (wl >> 2) + sq24(r - hl);
            for (int it = 0; it < C && lo < top; ++it) {
                const uint32_t wn = RW(lo + 1);
                const int hn = RH(lo + 1);
                const uint32_t bn = (wn >> 2) + sq24(r - hn);
                if (!(bn < bl))
                    break;
                ++lo;
                wl = wn;
                hl = hn;
                bl = bn;
            }
            bestB = bl;
            bestW = wl + (sq24(r - hl) << 2);
        };

        uint32_t cur[8], nxt[8];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            cur[k] = inp[(int64_t)min(k, n - 1) * stride + col];
        for (int i0 = 0; i0 < n; i0 += 8) {
#pragma unroll
            for (int k = 0; k < 8; ++k)
                nxt[k] = inp[(int64_t)min(i0 + 8 + k, n - 1) * stride + col];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int i = i0 + k;
                if (i >= n)
                    break;
                const uint32_t w = cur[k];
                if (w != QAI_WORD_INF && !ovf) {
                    const uint32_t g = w >> 2;
                    if (top > lo) {
                        uint32_t wt = RW(top);
                        int ht = RH(top);
                        for (int it = 0; it < C && top > lo; ++it) {
                            const uint32_t ws = RW(top - 1);
                            const int hs = RH(top - 1);
                            if (!remove_sel<SMALL>(ws >> 2, wt >> 2, g, hs, ht, i))
                                break;
                            --top;
                            wt = ws;
                            ht = hs;
                        }
                    }
                    if (top - lo + 1 >= C) {
                        ovf = true;
                    } else {
                        ++top;
                        RW(top) = w;
                        rhl[(top & (C - 1)) * 64] = (uint16_t)i;
                        if (e <= i)
                            refresh(e);
                    }
                }
                // emit the rows that are final for every column of the group
                for (int guard = 0; guard <= n; ++guard) {
                    const bool ok = (e <= i) && (ovf || bestB <= sq24(i + 1 - e));
                    const bool emit = (__ballot(ok) & gmask) == gmask;
                    if (__ballot(emit) == 0ull)
                        break;
                    if (emit) {
                        if (!ovf) {
                            outp[(int64_t)e * stride + lane] = bestW;
                            refresh(e + 1);
                        }
                        ++e;
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < 8; ++k)
                cur[k] = nxt[k];
        }
        // every remaining row is final
        for (; e < n; ++e) {
            if (!ovf) {
                outp[(int64_t)e * stride + lane] = bestW;
                refresh(e + 1);
            }
        }
#undef RW
#undef RH

        // columns whose live window outgrew the ring: exact outward search,
        // one column at a time by the whole wave, staged in the ring's LDS
        uint64_t om = __ballot(ovf && valid);
        const bool staged = n <= C * 64;
        while (om) {
            const int l = __ffsll((unsigned long long)om) - 1;
            om &= om - 1ull;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (staged)
                for (int r = lane; r < n; r += 64)
                    rw[r] = inp[(int64_t)r * stride + l];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (int p = lane; p < n; p += 64) {
                uint32_t best = staged ? rw[p] : inp[(int64_t)p * stride + l];
                for (int r = 1; r < n; ++r) {
                    const uint32_t r2 = (uint32_t)r * (uint32_t)r << 2;
                    if (r2 > (best | 3u))
                        break;
                    const int l0 = p - r, h0 = p + r;
                    if (l0 < 0 && h0 >= n)
                        break;
                    if (l0 >= 0) {
                        const uint32_t cand = word_add(staged ? rw[l0] : inp[(int64_t)l0 * stride + l], r2);
                        if ((cand >> 2) <= (best >> 2))
                            best = cand;
                    }
                    if (h0 < n) {
                        const uint32_t cand = word_add(staged ? rw[h0] : inp[(int64_t)h0 * stride + l], r2);
                        if ((cand >> 2) < (best >> 2))
                            best = cand;
                    }
                }
                outp[(int64_t)p * stride + l] = best;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

// Per-lane online envelope for payload-free words (the second EDT).  Same
// sweep as k_env_stream, but each lane emits its own rows: a row is final as
// soon as no later site can undercut it (its best value is at most the squared
// distance to the next unread row).  One emission attempt per row keeps the
// memory operations per row fixed (a lane with nothing final repeats its last
// store, so the compiler's counter waits stay exact); after every 8 rows, lanes
// whose live window nears the ring size emit all their final rows.  Ring
// entries are packed (g << hb) | row, checked on the host to fit 32 bits.
// Spare lanes of a partial tile shadow lane 0 (same column, same stores).
template <int AXIS, int C, bool SMALL, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_env_lane(EnvArgs a, int hb)
{
    __shared__ uint32_t ring[WPB * C * 64];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    uint32_t* const rl = ring + wv * C * 64 + lane;
    const int n = (int)((AXIS == 1) ? a.ny : a.nz);
    const int64_t stride = (AXIS == 1) ? a.nx : a.nx * a.ny;
    const int64_t nxb = (a.nx + 63) >> 6;
    const uint32_t hm = (1u << hb) - 1u;
    const uint64_t ngroups = (a.ntiles + WPB - 1) / WPB;
#define SLOT(k) (((k) & (C - 1)) * 64)

    for (uint64_t t = blockIdx.x; t < ngroups; t += gridDim.x) {
        const uint64_t tile = xcd_remap(t, ngroups) * WPB + wv;
        if (tile >= a.ntiles)
            continue;
        const int64_t xb = (int64_t)(tile % (uint64_t)nxb), o = (int64_t)(tile / (uint64_t)nxb);
        const int64_t x0 = xb * 64;
        const bool valid = x0 + lane < a.nx;
        const int64_t tb = ((AXIS == 1) ? o * a.nx * a.ny : o * a.nx) + x0;
        const uint32_t* __restrict__ inb = a.win + tb;
        uint32_t* const outb = a.w + tb;
        const uint32_t us = (uint32_t)stride;
        const uint32_t uc = valid ? (uint32_t)lane : 0u;

        int lo = 0, top = -1, e = 0;
        uint32_t be = 0xFFFFFFFFu;          // value at row e over the sites read so far
        uint32_t f0g = 0, f1g = 0, t0g = 0, t1g = 0, f2p = 0, t2p = 0;
        int f0h = 0, f1h = 0, t0h = 0, t1h = 0;
        bool ovf = false;
        uint32_t prow = 0, pval = QAI_WORD_INF;

        // advance the owner of row r (entries only leave from the front)
        auto front_to = [&](int r) {
            if (top < lo)
                return;
            uint32_t a0 = f0g + sq24(r - f0h);
            if (lo < top) {
                uint32_t a1 = f1g + sq24(r - f1h);
                if (a1 < a0) {
                    ++lo;
                    f0g = f1g; f0h = f1h; a0 = a1;
                    f1g = f2p >> hb; f1h = (int)(f2p & hm);
                    f2p = rl[SLOT(lo + 2)];
#pragma unroll 1
                    for (int it = 0; it < C && lo < top; ++it) {
                        a1 = f1g + sq24(r - f1h);
                        if (!(a1 < a0))
                            break;
                        ++lo;
                        f0g = f1g; f0h = f1h; a0 = a1;
                        f1g = f2p >> hb; f1h = (int)(f2p & hm);
                        f2p = rl[SLOT(lo + 2)];
                    }
                }
            }
            be = a0;
        };

        auto row_step = [&](int i, uint32_t w) {
            if (w != QAI_WORD_INF && !ovf) {
                const uint32_t g = w >> 2;
                if (top > lo && remove_sel<SMALL>(t1g, t0g, g, t1h, t0h, i)) {
                    --top;
                    t0g = t1g; t0h = t1h;
                    t1g = t2p >> hb; t1h = (int)(t2p & hm);
                    t2p = rl[SLOT(top - 2)];
#pragma unroll 1
                    for (int it = 0; it < C && top > lo; ++it) {
                        if (!remove_sel<SMALL>(t1g, t0g, g, t1h, t0h, i))
                            break;
                        --top;
                        t0g = t1g; t0h = t1h;
                        t1g = t2p >> hb; t1h = (int)(t2p & hm);
                        t2p = rl[SLOT(top - 2)];
                    }
                }
                if (top - lo + 1 >= C) {
                    ovf = true;
                } else {
                    ++top;
                    const uint32_t pk = (g << hb) | (uint32_t)i;
                    rl[SLOT(top)] = pk;
                    t2p = (t1g << hb) | (uint32_t)t1h;
                    t1g = t0g; t1h = t0h; t0g = g; t0h = i;
                    const uint32_t vi = g + sq24(e - i);
                    if (top == lo) {
                        f0g = g; f0h = i; be = vi;
                    } else {
                        if (top == lo + 1) { f1g = g; f1h = i; }
                        if (top == lo + 2) f2p = pk;
                        be = min(be, vi);
                    }
                }
            }
            const bool fin = !ovf && e <= i && top >= lo && be <= sq24(i + 1 - e);
            const uint32_t row = fin ? (uint32_t)e : prow;
            const uint32_t val = fin ? (be << 2) : pval;
            outb[row * us + uc] = val;
            prow = row;
            pval = val;
            e += fin ? 1 : 0;
            if (fin)
                front_to(e);
        };

        auto catch_up = [&](int i) {
#pragma unroll 1
            for (int it = 0; it < n; ++it) {
                const bool fin = !ovf && top - lo + 1 > C - 9 && e <= i && be <= sq24(i + 1 - e);
                if (__ballot(fin) == 0ull)
                    break;
                if (fin) {
                    outb[(uint32_t)e * us + uc] = be << 2;
                    ++e;
                    front_to(e);
                }
            }
        };

        // Full blocks of 16 rows, then the ragged tail.  Every prefetched word
        // is consumed before the catch-up loops, so no load is pending at
        // their entry (a loop with stores entered with a pending load costs a
        // wait for every outstanding memory operation).
        const int nfull = n & ~15;
        uint32_t A[8], B[8];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            A[k] = inb[(uint32_t)min(k, n - 1) * us + uc];
        for (int i0 = 0; i0 < nfull; i0 += 16) {
#pragma unroll
            for (int k = 0; k < 8; ++k)
                B[k] = inb[(uint32_t)(i0 + 8 + k) * us + uc];
#pragma unroll
            for (int k = 0; k < 8; ++k)
                row_step(i0 + k, A[k]);
            catch_up(i0 + 7);
#pragma unroll
            for (int k = 0; k < 8; ++k)
                A[k] = inb[(uint32_t)min(i0 + 16 + k, n - 1) * us + uc];
#pragma unroll
            for (int k = 0; k < 8; ++k)
                row_step(i0 + 8 + k, B[k]);
            catch_up(i0 + 15);
        }
#pragma unroll 1
        for (int i = nfull; i < n; ++i) {
            row_step(i, inb[(uint32_t)i * us + uc]);
            catch_up(i);
        }
        // every row left is final
#pragma unroll 1
        for (int it = 0; it < n; ++it) {
            const bool more = !ovf && e < n;
            if (__ballot(more) == 0ull)
                break;
            if (more) {
                outb[(uint32_t)e * us + uc] = (top >= lo) ? (be << 2) : QAI_WORD_INF;
                ++e;
                if (e < n)
                    front_to(e);
            }
        }
#undef SLOT

        // columns whose live window outgrew the ring: exact outward search,
        // one column at a time by the whole wave
        uint64_t om = __ballot(ovf && valid);
        while (om) {
            const int l = __ffsll((unsigned long long)om) - 1;
            om &= om - 1ull;
            for (int p = lane; p < n; p += 64) {
                uint32_t best = inb[(int64_t)p * stride + l];
                for (int r = 1; r < n; ++r) {
                    const uint32_t r2 = (uint32_t)r * (uint32_t)r << 2;
                    if (r2 > (best | 3u))
                        break;
                    const int l0 = p - r, h0 = p + r;
                    if (l0 < 0 && h0 >= n)
                        break;
                    if (l0 >= 0) {
                        const uint32_t cand = word_add(inb[(int64_t)l0 * stride + l], r2);
                        if ((cand >> 2) <= (best >> 2))
                            best = cand;
                    }
                    if (h0 < n) {
                        const uint32_t cand = word_add(inb[(int64_t)h0 * stride + l], r2);
                        if ((cand >> 2) < (best >> 2))
                            best = cand;
                    }
                }
                outb[(int64_t)p * stride + l] = best;
            }
        }
    }
}

// k_env_lane with stack entries kept as (c, h), c = g + h^2.  Maurer's
// removal test for sites u < v < w (Section III-B) then reads
//     (c_v - c_u)(h_w - h_v) - (c_w - c_v)(h_v - h_u) > 0,
// the same integer as c g_v - b g_u - a g_w - a b c (expand c_k = g_k + h_k^2),
// so with the differences of the top pair cached it costs two 24-bit
// multiplies; "the next entry is strictly better at row r" reads
// c_1 - c_0 < 2 r (h_1 - h_0).  A pop or a front step rebuilds its pair from
// one packed ring entry (c << hb) | h.  Loads and stores use 32-bit byte
// offsets into the tile (buffer instructions).  lane2_geometry checks that
// every value and product fits.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tile_rsrc(const void* p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

// BLK (y pass only): the result goes out in the blocked layout
// [z][y/4][x][y%4]: a lane collects its final rows in LDS and writes each
// group of four as one 16-byte store, a quarter of the write requests of
// single-word stores scattered over 64 rows.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// ovf_flag: when set, a wave with a column whose live window outgrew the
// ring raises it and leaves the whole pass to the banded pass gated on it;
// otherwise such columns take an exact outward search here.
template <int AXIS, int C, int WPB, bool BLK>
__device__ __forceinline__ void env_lane2(const EnvArgs& a, int hb, uint32_t* ring, uint32_t* stage,
                                          uint32_t* ovf_flag = nullptr)
{
    static_assert(!BLK || AXIS == 1, "blocked output is for the y pass");
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    uint32_t* const rl = ring + wv * C * 64 + lane;
    const int n = (int)((AXIS == 1) ? a.ny : a.nz);
    const int64_t stride = (AXIS == 1) ? a.nx : a.nx * a.ny;
    const int64_t nxb = (a.nx + 63) >> 6;
    const uint32_t hm = (1u << hb) - 1u;
    const uint64_t ngroups = (a.ntiles + WPB - 1) / WPB;
    const uint32_t us4 = (uint32_t)stride * 4u;
    const uint32_t span = (uint32_t)(n - 1) * us4 + 256u;
    const int64_t ny4 = (a.ny + 3) >> 2;
    uint32_t* const sl = stage + (BLK ? (wv * 64 + lane) * 4 : 0);
#define SLOT(k) (((k) & (C - 1)) * 64)

    // Tiles in dispatch order, not xcd_remap'd: a tile shares no cache line with
    // its neighbours, and the envelope's work follows the density of sites,
    // which changes from plane to plane: consecutive planes on different XCDs
    // spread the heavy ones.
    for (uint64_t t = blockIdx.x; t < ngroups; t += gridDim.x) {
        const uint64_t tile = t * WPB + wv;
        if (tile >= a.ntiles)
            continue;
        const int64_t xb = (int64_t)(tile % (uint64_t)nxb), o = (int64_t)(tile / (uint64_t)nxb);
        const int64_t x0 = xb * 64;
        const bool valid = x0 + lane < a.nx;
        const int64_t tb = ((AXIS == 1) ? o * a.nx * a.ny : o * a.nx) + x0;
        // blocked: the tile's words start at (o ny4 nx + x0) 4; row group k
        // of lane l lies (k nx + l) 16 bytes further
        const int64_t tbo = BLK ? (o * ny4 * a.nx + x0) * 4 : tb;
        const uint32_t span_out = BLK ? (uint32_t)(((ny4 - 1) * a.nx + 64) * 16) : span;
        const __amdgpu_buffer_rsrc_t rin = tile_rsrc(a.win + tb, span);
        const __amdgpu_buffer_rsrc_t rout = tile_rsrc(a.w + tbo, span_out);
        const uint32_t vo = (valid ? (uint32_t)lane : 0u) * 4u;
        const uint32_t bo = (valid ? (uint32_t)lane : 0u) * 16u;
        const uint32_t bstep = (uint32_t)a.nx * 16u;

        // blocked: the final value v of a row goes to the lane's stage, and out
        // with the fourth row of its group or the last row of the line
        auto emit_blk = [&](int row, uint32_t v) {
            sl[row & 3] = v;
            if ((row & 3) == 3 || row == n - 1) {
                const u32x4 q = *reinterpret_cast<const u32x4*>(sl);
                __builtin_amdgcn_raw_buffer_store_b128(q, rout, bo + __umul24((uint32_t)(row >> 2), bstep), 0, 0);
            }
        };

        int lo = 0, top = -1;
        int c0 = 0, h0 = 0, dc = 0, dh = 0;     // top entry, difference to the one below
        uint32_t t2p = 0;                        // packed entry two below the top
        int fc0 = 0, fh0 = 0, dfc = 0, dfh = 0;  // front entry, difference to the next
        uint32_t f2p = 0;                        // packed entry two after the front
        int e = 0;                               // next row to emit
        uint32_t be = 0xFFFFFFFFu;               // value at row e over the sites read so far
        uint32_t eoff = vo, poff = vo, pval = QAI_WORD_INF;
        bool ovf = false;

        // (the loop tests below evaluate both operands, no short circuit: the
        // second reads entries outside the live window once the first fails,
        // whose values are then unused, and a branch per test costs more
        // scalar and branch instructions than the arithmetic it skips)
        // the owner of row e: step while the next entry is strictly better
        // (24-bit products: lane2_geometry keeps lines below 1024 rows, so
        // 2 e dfh and e (e - 2 fh0) fit; a 32-bit multiply costs four times as
        // much.  2 e and dfh are never negative: the unsigned form needs no
        // sign extension of its operands)
        auto walk = [&]() {
            const int e2 = 2 * e;
            if ((lo < top) & (dfc < (int)__umul24((uint32_t)e2, (uint32_t)dfh))) {
#pragma unroll 1
                do {
                    ++lo;
                    fc0 += dfc;
                    fh0 += dfh;
                    dfc = (int)(f2p >> hb) - fc0;
                    dfh = (int)(f2p & hm) - fh0;
                    f2p = rl[SLOT(lo + 2)];
                } while ((lo < top) & (dfc < (int)__umul24((uint32_t)e2, (uint32_t)dfh)));
            }
            be = (uint32_t)(fc0 + __mul24(e, e - 2 * fh0));
        };

        // A lane whose live window fills the ring sets ovf and holds be at
        // "none" from then on: its column is redone (the banded pass or the
        // outward search below), so its ring may be overwritten.  "Row e is
        // final" then reads be <= (i + 1 - e)^2 alone: a finite be means a
        // site was read (top >= lo), and e = i + 1 never passes (its owner
        // lies at least a row away).
        auto row_step = [&](int i, uint32_t w) {
            if ((w != QAI_WORD_INF) & !ovf) { // one branch for both conditions
                const int g = (int)(w >> 2);
                const int cw = g + i * i;
                bool rm = (top > lo) & (__mul24(dc, i - h0) > __mul24(cw - c0, dh));
#pragma unroll 1
                while (rm) {
                    --top;
                    c0 -= dc;
                    h0 -= dh;
                    dc = c0 - (int)(t2p >> hb);
                    dh = h0 - (int)(t2p & hm);
                    t2p = rl[SLOT(top - 2)];
                    rm = (top > lo) & (__mul24(dc, i - h0) > __mul24(cw - c0, dh));
                }
                ovf = top - lo + 1 >= C;
                t2p = rl[SLOT(top - 1)];
                ++top;
                const uint32_t pk = ((uint32_t)cw << hb) | (uint32_t)i;
                rl[SLOT(top)] = pk;
                dc = cw - c0;
                dh = i - h0;
                c0 = cw;
                h0 = i;
                be = ovf ? 0xFFFFFFFFu : min(be, (uint32_t)(g + __mul24(e - i, e - i)));
                const int ws = top - lo;
                fc0 = ws == 0 ? cw : fc0;
                fh0 = ws == 0 ? i : fh0;
                dfc = ws == 1 ? dc : dfc;
                dfh = ws == 1 ? dh : dfh;
                f2p = ws == 2 ? pk : f2p;
            }
            // one emission slot per row (unblocked: a lane with nothing final
            // repeats its last store, so the memory operations per row stay fixed)
            const int q = i + 1 - e; // 0 <= q <= i + 1
            const bool fin = be <= __umul24((uint32_t)q, (uint32_t)q);
            if (BLK) {
                if (fin)
                    emit_blk(e, be << 2);
            } else {
                const uint32_t off = fin ? eoff : poff;
                const uint32_t val = fin ? (be << 2) : pval;
                __builtin_amdgcn_raw_buffer_store_b32(val, rout, off, 0, 0);
                poff = off;
                pval = val;
            }
            if (fin) {
                ++e;
                eoff += us4;
                walk();
            }
        };

        // lanes whose live window nears the ring size emit all their final rows
        auto catch_up = [&](int i) {
#pragma unroll 1
            for (int it = 0; it < n; ++it) {
                const int q = i + 1 - e;
                const bool fin = top - lo + 1 > C - 9 && be <= __umul24((uint32_t)q, (uint32_t)q);
                if (__ballot(fin) == 0ull)
                    break;
                if (fin) {
                    if (BLK)
                        emit_blk(e, be << 2);
                    else
                        __builtin_amdgcn_raw_buffer_store_b32(be << 2, rout, eoff, 0, 0);
                    ++e;
                    eoff += us4;
                    walk();
                }
            }
        };

        // full blocks of 16 rows (every prefetched word used before the
        // catch-up loops), then the tail
        const int nfull = n & ~15;
        uint32_t A[8], B[8];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            A[k] = __builtin_amdgcn_raw_buffer_load_b32(rin, vo, (uint32_t)min(k, n - 1) * us4, 0);
        for (int i0 = 0; i0 < nfull; i0 += 16) {
#pragma unroll
            for (int k = 0; k < 8; ++k)
                B[k] = __builtin_amdgcn_raw_buffer_load_b32(rin, vo, (uint32_t)(i0 + 8 + k) * us4, 0);
#pragma unroll
            for (int k = 0; k < 8; ++k)
                row_step(i0 + k, A[k]);
            catch_up(i0 + 7);
#pragma unroll
            for (int k = 0; k < 8; ++k)
                A[k] = __builtin_amdgcn_raw_buffer_load_b32(rin, vo, (uint32_t)min(i0 + 16 + k, n - 1) * us4, 0);
#pragma unroll
            for (int k = 0; k < 8; ++k)
                row_step(i0 + 8 + k, B[k]);
            catch_up(i0 + 15);
        }
#pragma unroll 1
        for (int i = nfull; i < n; ++i) {
            row_step(i, __builtin_amdgcn_raw_buffer_load_b32(rin, vo, (uint32_t)i * us4, 0));
            catch_up(i);
        }
        // every row left is final
#pragma unroll 1
        for (int it = 0; it < n; ++it) {
            const bool more = !ovf && e < n;
            if (__ballot(more) == 0ull)
                break;
            if (more) {
                const uint32_t v = (top >= lo) ? (be << 2) : QAI_WORD_INF;
                if (BLK)
                    emit_blk(e, v);
                else
                    __builtin_amdgcn_raw_buffer_store_b32(v, rout, eoff, 0, 0);
                ++e;
                eoff += us4;
                if (e < n && top >= lo)
                    walk();
            }
        }
#undef SLOT

        // columns whose live window outgrew the ring: exact outward search,
        // one column at a time by the whole wave
        const uint32_t* __restrict__ inb = a.win + tb;
        uint32_t* const outb = a.w + tbo;
        uint64_t om = __ballot(ovf && valid);
        if (ovf_flag && om) {
            if (lane == 0)
                atomicOr(ovf_flag, 1u);
            om = 0ull;
        }
        while (om) {
            const int l = __ffsll((unsigned long long)om) - 1;
            om &= om - 1ull;
            for (int p = lane; p < n; p += 64) {
                uint32_t best = inb[(int64_t)p * stride + l];
                for (int r = 1; r < n; ++r) {
                    const uint32_t r2 = (uint32_t)r * (uint32_t)r << 2;
                    if (r2 > (best | 3u))
                        break;
                    const int l0 = p - r, h1 = p + r;
                    if (l0 < 0 && h1 >= n)
                        break;
                    if (l0 >= 0) {
                        const uint32_t cand = word_add(inb[(int64_t)l0 * stride + l], r2);
                        if ((cand >> 2) <= (best >> 2))
                            best = cand;
                    }
                    if (h1 < n) {
                        const uint32_t cand = word_add(inb[(int64_t)h1 * stride + l], r2);
                        if ((cand >> 2) < (best >> 2))
                            best = cand;
                    }
                }
                if (BLK)
                    outb[((int64_t)(p >> 2) * a.nx + l) * 4 + (p & 3)] = best;
                else
                    outb[(int64_t)p * stride + l] = best;
            }
        }
    }
}

template <int AXIS, int C, int WPB, bool BLK>
__global__ __launch_bounds__(64 * WPB) void k_env_lane2(EnvArgs a, int hb)
{
    __shared__ uint32_t ring[WPB * C * 64];
    __shared__ __align__(16) uint32_t stage[BLK ? WPB * 64 * 4 : 4];
    env_lane2<AXIS, C, WPB, BLK>(a, hb, ring, stage);
}

// The second EDT's y pass by the per-lane envelope.  Ahead of the
// needed-voxel search its output layout is chosen on the device
// (blocked_layout) from the first seed pass's B1 estimate, blocked where
// there is none (b1count null); ahead of a whole z pass (natural) it is the
// natural layout.
template <int C, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_env_lane2_y(EnvArgs a, int hb, const unsigned long long* b1count,
                                                          uint32_t* ovf_flag, bool natural)
{
    __shared__ uint32_t ring[WPB * C * 64];
    __shared__ __align__(16) uint32_t stage[WPB * 64 * 4];
    if (!natural && (!b1count || blocked_layout(b1count, (uint64_t)(a.nx * a.ny * a.nz))))
        env_lane2<1, C, WPB, true>(a, hb, ring, stage, ovf_flag);
    else
        env_lane2<1, C, WPB, false>(a, hb, ring, stage, ovf_flag);
}

// A whole z pass of the second EDT by the per-lane envelope, its
// overflowing columns handed to the banded pass as in k_env_lane2_y.
// only_sparse: when set, the pass runs only where sparse_b1 holds.
template <int C, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_env_lane2_z(EnvArgs a, int hb, uint32_t* ovf_flag,
                                                          const unsigned long long* only_sparse)
{
    __shared__ uint32_t ring[WPB * C * 64];
    __shared__ __align__(16) uint32_t stage[4];
    if (only_sparse && !sparse_b1(only_sparse, (uint64_t)(a.nx * a.ny * a.nz)))
        return;
    env_lane2<2, C, WPB, false>(a, hb, ring, stage, ovf_flag);
}

__global__ void k_clear(uint32_t* p, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = 0u;
}

// ------------------------------------------------------------- launchers
static uint32_t grid_cap(uint64_t units, uint64_t cap)
{
    uint64_t g = units < cap ? units : cap;
    if (g >= QAI_NUM_XCD)
        g -= g % QAI_NUM_XCD; // a multiple of 8 keeps each workgroup on one XCD's range
    return (uint32_t)(g ? g : 1);
}

void default_tuning(Tuning& t)
{
    for (int i = 0; i < 3; ++i) {
        t.env_tx_log2[i] = -1;
        t.env_algo[i] = -1; // chosen per pass from its parallelism (see resolve_algo)
        t.edt1_algo[i] = -1;
        t.stream_cap[i] = 32;
        t.edt1_cap[i] = 16;
    }
    t.env_threads = 256;
    t.seed_ty = 0;
    t.seed_tz = 16;
    t.force_wide = 0;
}

static hipError_t launch_seed_lines(int mode, const SeedArgs& in, hipStream_t s)
{
    SeedArgs a = in;
    const int64_t nch = (a.nx + 63) / 64;
    const size_t per_wave = ((mode == 0 ? (size_t)nch * 64 : 0) + (size_t)nch * 12 + 15) & ~(size_t)15;
    int waves = 4;
    while (waves > 1 && per_wave * waves > 64 * 1024)
        waves >>= 1;
    a.waves = waves;
    const int64_t lines = a.ny * a.nz;
    a.ngroups = (uint64_t)((lines + waves - 1) / waves);
    const uint32_t grid = grid_cap(a.ngroups, 1u << 20);
    const size_t shm = per_wave * waves;
    if (mode == 0)
        return launch_checked(k_seed_xscan<0>, dim3(grid), dim3(64 * waves), shm, s, a);
    else
        return launch_checked(k_seed_xscan<1>, dim3(grid), dim3(64 * waves), shm, s, a);
}

static size_t slab_bytes(int64_t nx, int ty, int rows, int planes)
{
    const int64_t nch = (nx + 63) / 64;
    const size_t ring = ((size_t)planes * rows * nx * 4 + 15) & ~(size_t)15;
    return ring + (size_t)ty * nch * (64 + 8 + 4) + 64;
}

template <int MODE, int V, int P = 1, int WPB = 8>
static hipError_t launch_seed_lane_t(const SeedArgs& in, int tz, hipStream_t s)
{
    const bool taps = (MODE == 0) ? (in.tq || in.tb1 || in.tsb) : (in.ts || in.td1 || in.tb2);
    constexpr int LP = WPB / P;
    constexpr int VW4 = (V % 4 == 0) ? 4 : 1, VW2 = (V % 2 == 0) ? 2 : 1;
    if (in.nx > 64 * V * P)
        return hipErrorInvalidValue;
    SlabArgs A;
    A.s = in;
    A.ty = LP;
    A.rows = LP + 2;
    A.planes = 3;
    A.tz = tz;
    A.nby = (in.ny + LP - 1) / LP;
    A.nbz = (in.nz + tz - 1) / tz;
    const uint32_t grid = grid_cap((uint64_t)(A.nby * A.nbz), 1u << 20);
    const uintptr_t al = (uintptr_t)((MODE == 0) ? (const void*)in.xq : (const void*)in.w1) | (uintptr_t)in.wout;
    const dim3 g(grid), b(64 * WPB);
    if (taps)
        return launch_checked(k_seed_lane<MODE, V, WPB, 1, true, P>, g, b, 0, s, A);
    else if (V % 4 == 0 && in.nx % 4 == 0 && al % 16 == 0)
        return launch_checked(k_seed_lane<MODE, V, WPB, VW4, false, P>, g, b, 0, s, A);
    else if (V % 2 == 0 && in.nx % 2 == 0 && al % 8 == 0)
        return launch_checked(k_seed_lane<MODE, V, WPB, VW2, false, P>, g, b, 0, s, A);
    else
        return launch_checked(k_seed_lane<MODE, V, WPB, 1, false, P>, g, b, 0, s, A);
}

template <int MODE>
static hipError_t launch_seed_lane(const SeedArgs& in, int tz, hipStream_t s)
{
    // lines of 513..4096 voxels: two, four or eight waves per line (eight in
    // workgroups of sixteen waves: two lines each)
    if (in.nx > 2048)
        return launch_seed_lane_t<MODE, 8, 8, 16>(in, tz, s);
    if (in.nx > 1024)
        return launch_seed_lane_t<MODE, 8, 4>(in, tz, s);
    // step A in workgroups of four waves from four voxels per lane up: each
    // plane's barrier waits for fewer waves (seed1 on 512^3 290 -> 250 us,
    // 100x500x500 104 -> 81, 384^3 151 -> 127, 96x256x768 77 -> 66,
    // 200x300x300 80 -> 74 us; level on 128x128x1024 and 300x400x400).  Step C
    // keeps eight (512^3: 216 against 229 us; 384^3 118 against 129 us).
    constexpr int W4 = MODE == 0 ? 4 : 8;
    if (in.nx > 512)
        return launch_seed_lane_t<MODE, 8, 2, W4>(in, tz, s);
    switch ((int)((in.nx + 63) / 64)) {
    case 1: return launch_seed_lane_t<MODE, 1>(in, tz, s);
    case 2: return launch_seed_lane_t<MODE, 2>(in, tz, s);
    case 3: return launch_seed_lane_t<MODE, 3>(in, tz, s);
    case 4: return launch_seed_lane_t<MODE, 4, 1, W4>(in, tz, s);
    case 5: return launch_seed_lane_t<MODE, 5, 1, W4>(in, tz, s);
    case 6: return launch_seed_lane_t<MODE, 6, 1, W4>(in, tz, s);
    case 7: return launch_seed_lane_t<MODE, 7, 1, W4>(in, tz, s);
    default: return launch_seed_lane_t<MODE, 8, 1, W4>(in, tz, s);
    }
}

// Step A from coded indices (k_seed_lane mode 2): lines whose lanes each hold
// a whole share of one 32-voxel segment: up to 512 voxels with ceil(nx / 64)
// dividing 32, and 513..2048 voxels (eight voxels per lane, two or four waves
// per line; eight waves would leave the decode too few registers).
constexpr int64_t kCodedSeedMaxX = 2048;
bool coded_seed_supported(int64_t nx)
{
    const int64_t v = (nx + 63) / 64;
    return (nx <= 512 && (v == 1 || v == 2 || v == 4 || v == 8)) || (nx > 512 && nx <= kCodedSeedMaxX);
}

template <int V, int P = 1, int WPB = 8>
static hipError_t launch_seed_coded_t(const SeedArgs& in, int tz, hipStream_t s)
{
    constexpr int LP = WPB / P;
    constexpr int VW4 = (V % 4 == 0) ? 4 : 1, VW2 = (V % 2 == 0) ? 2 : 1;
    if (in.nx > 64 * V * P)
        return hipErrorInvalidValue;
    SlabArgs A;
    A.s = in;
    A.ty = LP;
    A.rows = LP + 2;
    A.planes = 3;
    A.tz = tz;
    A.nby = (in.ny + LP - 1) / LP;
    A.nbz = (in.nz + tz - 1) / tz;
    const uint32_t grid = grid_cap((uint64_t)(A.nby * A.nbz), 1u << 20);
    const uintptr_t al = (uintptr_t)in.xout | (uintptr_t)in.wout;
    const dim3 g(grid), b(64 * WPB);
    if (V % 4 == 0 && in.nx % 4 == 0 && al % 16 == 0)
        return launch_checked(k_seed_lane<2, V, WPB, VW4, false, P>, g, b, 0, s, A);
    if (V % 2 == 0 && in.nx % 2 == 0 && al % 8 == 0)
        return launch_checked(k_seed_lane<2, V, WPB, VW2, false, P>, g, b, 0, s, A);
    return launch_checked(k_seed_lane<2, V, WPB, 1, false, P>, g, b, 0, s, A);
}

hipError_t launch_seed_coded(const SeedArgs& in, int tz, hipStream_t s)
{
    if (in.nx > kCodedSeedMaxX)
        return hipErrorInvalidValue;
    if (in.nx > 1024)
        return launch_seed_coded_t<8, 4>(in, tz, s);
    if (in.nx > 512)
        return launch_seed_coded_t<8, 2>(in, tz, s);
    switch ((int)((in.nx + 63) / 64)) {
    case 1: return launch_seed_coded_t<1>(in, tz, s);
    case 2: return launch_seed_coded_t<2>(in, tz, s);
    case 4: return launch_seed_coded_t<4>(in, tz, s);
    case 8: return launch_seed_coded_t<8, 1, 4>(in, tz, s); // four waves, as the plain step A
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_seed(int mode, const SeedArgs& in, hipStream_t s, int want_ty, int want_tz)
{
    if (want_ty < 0)
        return launch_seed_lines(mode, in, s); // one x-line per wave, neighbours through the caches
    if (in.nx <= kSeedLaneMaxX && want_ty <= 0) {
        const int tz = in.nz > 1 ? (want_tz > 0 ? want_tz : 16) : 1;
        return mode == 0 ? launch_seed_lane<0>(in, tz, s) : launch_seed_lane<1>(in, tz, s);
    }
    const int planes = in.nz > 1 ? 3 : 1;
    if (want_ty <= 0) {
        // one line per workgroup, split over eight wavefronts
        constexpr int SEG = 8;
        const int rows = in.ny > 1 ? 3 : 1;
        const int nch = (int)((in.nx + 63) / 64);
        const size_t lds = (((size_t)planes * rows * in.nx * 4 + 15) & ~(size_t)15) +
                           (((size_t)nch * 64 + 15) & ~(size_t)15) + (size_t)nch * 12;
        if (lds <= 96 * 1024 && nch >= SEG) {
            SlabArgs A;
            A.s = in;
            A.ty = 1;
            A.rows = rows;
            A.planes = planes;
            A.tz = in.nz > 1 ? (want_tz > 0 ? want_tz : 16) : 1;
            A.nby = in.ny;
            A.nbz = (in.nz + A.tz - 1) / A.tz;
            const uint32_t grid = grid_cap((uint64_t)(A.nby * A.nbz), 1u << 20);
            if (mode == 0)
                return launch_checked(k_seed_seg<0, SEG>, dim3(grid), dim3(64 * SEG), lds, s, A);
            else
                return launch_checked(k_seed_seg<1, SEG>, dim3(grid), dim3(64 * SEG), lds, s, A);
        }
    }
    int ty = want_ty > 0 ? want_ty : 4;
    if (in.ny == 1)
        ty = 1;
    auto rows_of = [&](int t) { return in.ny > 1 ? t + 2 : 1; };
    while (ty > 1 && slab_bytes(in.nx, ty, rows_of(ty), planes) > 96 * 1024)
        ty >>= 1;
    if (slab_bytes(in.nx, ty, rows_of(ty), planes) > 96 * 1024)
        return launch_seed_lines(mode, in, s); // very long x-lines: one line per wave
    SlabArgs A;
    A.s = in;
    A.ty = ty;
    A.rows = rows_of(ty);
    A.planes = planes;
    A.tz = in.nz > 1 ? (want_tz > 0 ? want_tz : 16) : 1;
    A.nby = (in.ny + ty - 1) / ty;
    A.nbz = (in.nz + A.tz - 1) / A.tz;
    const size_t lds = slab_bytes(in.nx, ty, A.rows, planes);
    const uint32_t grid = grid_cap((uint64_t)(A.nby * A.nbz), 1u << 20);
    const int threads = 64 * (ty < 4 ? 4 : ty);
    if (mode == 0)
        return launch_checked(k_seed_slab<0>, dim3(grid), dim3(threads), lds, s, A);
    else
        return launch_checked(k_seed_slab<1>, dim3(grid), dim3(threads), lds, s, A);
}

static int default_tx_log2(int64_t n)
{
    // windowed variant: keep the staged tile within 32 KB
    int l = 4;
    while (l > 0 && (n << l) * 4 > 32 * 1024)
        --l;
    return l;
}

template <int AXIS, int M>
static hipError_t launch_band2_t(EnvArgs a, int lb, size_t lds, int threads, uint32_t grid, hipStream_t s)
{
    static bool attr_done = false;
    if (lds > 64 * 1024 && !attr_done) {
        hipError_t e = hipFuncSetAttribute((const void*)k_env_band2<AXIS, M>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess)
            return e;
        attr_done = true;
    }
    return launch_checked(k_env_band2<AXIS, M>, dim3(grid), dim3(threads), lds, s, a, lb);
}

template <int AXIS>
static hipError_t launch_band2_m(EnvArgs a, int M, int lb, size_t lds, int threads, uint32_t grid, hipStream_t s)
{
    switch (M) {
    case 8: return launch_band2_t<AXIS, 8>(a, lb, lds, threads, grid, s);
    case 16: return launch_band2_t<AXIS, 16>(a, lb, lds, threads, grid, s);
    default: return launch_band2_t<AXIS, 32>(a, lb, lds, threads, grid, s);
    }
}

// Geometry of the wave-per-column banded variant: bands of M = max(8, 2^k)
// positions with at most 64 bands, B = 2^lb bands per column, Tx columns per
// tile (the LDS image is 8 bytes per padded position).
static void band2_geometry(int n, int want_txl, int& M, int& lb, int& txl, size_t& lds)
{
    M = 8;
    while (M * 64 < n)
        M <<= 1;
    int nb = (n + M - 1) / M;
    lb = 0;
    while ((1 << lb) < nb)
        ++lb;
    const int B = 1 << lb;
    txl = want_txl >= 0 ? want_txl : 3;
    while ((B << txl) > 1024)
        --txl;
    while (txl > 0 && (size_t)(B * (M + 1) + 1) * (1 << txl) * 8 > 80 * 1024)
        --txl;
    while ((B << txl) < 64)
        ++txl;
    lds = (size_t)(B * (M + 1) + 1) * (1 << txl) * 8;
}

static hipError_t launch_band2(int axis, EnvArgs a, const Tuning& t, hipStream_t s)
{
    const int n = (int)(axis == 1 ? a.ny : a.nz);
    int M, lb, txl;
    size_t lds;
    band2_geometry(n, t.env_tx_log2[axis], M, lb, txl, lds);
    a.tx_log2 = txl;
    const int64_t nxb = (a.nx + (1 << txl) - 1) >> txl;
    a.ntiles = (uint64_t)(nxb * (axis == 1 ? a.nz : a.ny));
    // a gated launch (usually not needed) keeps its grid small: every block
    // starts only to read the gate
    const uint32_t grid = grid_cap(a.ntiles, a.gate ? 2048u : (1u << 20));
    const int threads = (1 << lb) << txl;
    if (axis == 1)
        return launch_band2_m<1>(a, M, lb, lds, threads, grid, s);
    return launch_band2_m<2>(a, M, lb, lds, threads, grid, s);
}

template <int AXIS, int C>
static hipError_t launch_stream_t(EnvArgs a, bool force_wide, hipStream_t s)
{
    // LDS ring: 6 bytes x C entries x 64 lanes per wave
    const int waves = C >= 32 ? 1 : 2;
    const int64_t nxb = (a.nx + 63) >> 6;
    a.ntiles = (uint64_t)(nxb * (AXIS == 1 ? a.nz : a.ny));
    const uint64_t groups = (a.ntiles + waves - 1) / waves;
    const size_t lds = (size_t)waves * C * 64 * 6;
    const int64_t n = AXIS == 1 ? a.ny : a.nz;
    // site values are squared distances within the lower dimensions
    const int64_t gmax = (a.nx - 1) * (a.nx - 1) + (AXIS == 2 ? (a.ny - 1) * (a.ny - 1) : 0);
    const bool small =
        !force_wide && n < 4096 && gmax < (1 << 24) && n * gmax + n * n * n / 4 < (int64_t)1 << 31;
    const dim3 grid(grid_cap(groups, 1u << 20)), blk(64 * waves);
    if (small)
        return launch_checked(k_env_stream<AXIS, C, true>, grid, blk, lds, s, a);
    else
        return launch_checked(k_env_stream<AXIS, C, false>, grid, blk, lds, s, a);
}

// Ring entries pack (g << hb) | row into 32 bits: hb covers the rows of the
// pass, g the largest squared distance the previous passes can produce.
static bool lane_geometry(int axis, const EnvArgs& a, int& hb, bool& small)
{
    const int64_t n = axis == 1 ? a.ny : a.nz;
    const int64_t gmax = (a.nx - 1) * (a.nx - 1) + (axis == 2 ? (a.ny - 1) * (a.ny - 1) : 0);
    hb = 1;
    while (((int64_t)1 << hb) < n)
        ++hb;
    small = n < 4096 && gmax < (1 << 24) && n * gmax + n * n * n / 4 < (int64_t)1 << 31;
    return n < 65536 && hb < 32 && gmax < ((int64_t)1 << (32 - hb));
}

// k_env_lane2 is exact when, with c_max = g_max + (n - 1)^2: packed entries
// fit 32 bits (c_max < 2^(32 - hb)), every multiplied operand fits 24 bits
// (c_max < 2^23), the two products of the removal test and their difference
// stay in int32 (c_max n < 2^30), and the tile's byte span fits a buffer.
static bool lane2_geometry(int axis, const EnvArgs& a, int& hb)
{
    const int64_t n = axis == 1 ? a.ny : a.nz;
    const int64_t stride = axis == 1 ? a.nx : a.nx * a.ny;
    const int64_t gmax = (a.nx - 1) * (a.nx - 1) + (axis == 2 ? (a.ny - 1) * (a.ny - 1) : 0);
    const int64_t cmax = gmax + (n - 1) * (n - 1);
    hb = 1;
    while (((int64_t)1 << hb) < n)
        ++hb;
    return hb < 24 && cmax < ((int64_t)1 << (32 - hb)) && cmax < ((int64_t)1 << 23) &&
           cmax * n < ((int64_t)1 << 30) && (n - 1) * stride * 4 + 256 < ((int64_t)1 << 31);
}

template <int AXIS, bool BLK = false>
static hipError_t launch_lane2_t(EnvArgs a, int hb, hipStream_t s)
{
    constexpr int WPB = 4;
    const int64_t nxb = (a.nx + 63) >> 6;
    a.ntiles = (uint64_t)(nxb * (AXIS == 1 ? a.nz : a.ny));
    const uint64_t groups = (a.ntiles + WPB - 1) / WPB;
    return launch_checked(k_env_lane2<AXIS, 32, WPB, BLK>, dim3(grid_cap(groups, 1u << 20)), dim3(64 * WPB), 0, s, a,
                       hb);
}

// Ring entries per lane: 32 where the pass has more than 2048 tiles (the
// ring's LDS then limits a CU to 16 waves, the occupancy that pays at 512^3:
// 664 us against 824 us with 64 entries and, with 16, an overflow in some
// column), 64 below (no more waves to hold; fewer catch-ups and overflows:
// 256^3 at rel. bound 5e-3, 222 -> 188 us).
static hipError_t launch_lane2_y(EnvArgs a, int hb, const unsigned long long* b1count, uint32_t* ovf_flag,
                                 bool natural, hipStream_t s)
{
    constexpr int WPB = 4;
    const int64_t nxb = (a.nx + 63) >> 6;
    a.ntiles = (uint64_t)(nxb * a.nz);
    const uint64_t groups = (a.ntiles + WPB - 1) / WPB;
    const dim3 grid(grid_cap(groups, 1u << 20)), blk(64 * WPB);
    if (a.ntiles <= 2048)
        return launch_checked(k_env_lane2_y<64, WPB>, grid, blk, 0, s, a, hb, b1count, ovf_flag, natural);
    return launch_checked(k_env_lane2_y<32, WPB>, grid, blk, 0, s, a, hb, b1count, ovf_flag, natural);
}

// (ring entries as for the y pass)
static hipError_t launch_lane2_z(EnvArgs a, int hb, uint32_t* ovf_flag, const unsigned long long* only_sparse,
                                 hipStream_t s)
{
    constexpr int WPB = 4;
    const int64_t nxb = (a.nx + 63) >> 6;
    a.ntiles = (uint64_t)(nxb * a.ny);
    const uint64_t groups = (a.ntiles + WPB - 1) / WPB;
    const dim3 grid(grid_cap(groups, 1u << 20)), blk(64 * WPB);
    if (a.ntiles <= 2048)
        return launch_checked(k_env_lane2_z<64, WPB>, grid, blk, 0, s, a, hb, ovf_flag, only_sparse);
    return launch_checked(k_env_lane2_z<32, WPB>, grid, blk, 0, s, a, hb, ovf_flag, only_sparse);
}

template <int AXIS>
static hipError_t launch_lane_t(EnvArgs a, int hb, bool small, hipStream_t s)
{
    constexpr int WPB = 4;
    const int64_t nxb = (a.nx + 63) >> 6;
    a.ntiles = (uint64_t)(nxb * (AXIS == 1 ? a.nz : a.ny));
    const uint64_t groups = (a.ntiles + WPB - 1) / WPB;
    const dim3 grid(grid_cap(groups, 1u << 20)), blk(64 * WPB);
    if (small)
        return launch_checked(k_env_lane<AXIS, 32, true, WPB>, grid, blk, 0, s, a, hb);
    else
        return launch_checked(k_env_lane<AXIS, 32, false, WPB>, grid, blk, 0, s, a, hb);
}

template <int AXIS>
static hipError_t launch_swin_t(EnvArgs a, hipStream_t s)
{
    constexpr int WPB = 4;
    const int64_t nxb = (a.nx + 63) >> 6;
    a.ntiles = (uint64_t)(nxb * (AXIS == 1 ? a.nz : a.ny));
    const uint64_t groups = (a.ntiles + WPB - 1) / WPB;
    return launch_checked(k_env_swin<AXIS, WPB>, dim3(grid_cap(groups, 1u << 20)), dim3(64 * WPB), 0, s, a);
}

// ----------------------------------------------- first EDT, y and z at once
// After the x pass, the first EDT's y and z passes together give, at each
// voxel, the minimum over (z', y') of G(z', y') + (z - z')^2 + (y - y')^2 (G:
// the x-pass distance in row (z', y')), the separable passes keeping among
// equal values the lowest z', then the lowest y' (Algorithm 1's strict
// comparisons along each axis): the lexicographically smallest (z', y').
// B1 is dense and its distances short, so one pass takes that minimum over a
// disc of offsets directly: a voxel with G = best = b is final once every
// offset with dz^2 + dy^2 <= b has been compared (any other candidate costs
// more than b), and offsets are taken in order of dz^2 + dy^2.  A voxel whose
// best exceeds the disc (radius^2 YZ_R2), or has no site in it, raises *wide;
// the separable passes then run after it (gated on *wide) and recompute the
// whole field exactly, and blocks that start after the flag is up stop at
// once (sparse B1: the pass costs little more than the separable passes).
constexpr int YZ_R = 12, YZ_R2 = YZ_R * YZ_R;
struct YzTable {
    uint32_t e[512]; // (dz^2 + dy^2) << 16 | (dz + 128) << 8 | (dy + 128), ascending; padded with all ones
    int n;           // entries, padding excluded
};
constexpr YzTable make_yz_table()
{
    YzTable t{};
    int n = 0;
    for (int dz = -YZ_R; dz <= YZ_R; ++dz)
        for (int dy = -YZ_R; dy <= YZ_R; ++dy) {
            const int d2 = dz * dz + dy * dy;
            if (d2 == 0 || d2 > YZ_R2)
                continue;
            const uint32_t v = ((uint32_t)d2 << 16) | ((uint32_t)(dz + 128) << 8) | (uint32_t)(dy + 128);
            int k = n++;
            while (k > 0 && t.e[k - 1] > v) {
                t.e[k] = t.e[k - 1];
                --k;
            }
            t.e[k] = v;
        }
    t.n = n;
    while (n % 4)
        t.e[n++] = 0xFFFFFFFFu;
    return t;
}
__constant__ YzTable c_yz = make_yz_table();

// Four consecutive voxels of a row per quad (nx a multiple of 4).  A block
// takes 512 quads at a time, two per thread 256 apart, their loads in flight
// together (against four per thread: 256x384x384 65 -> 58 us, 512^3 level;
// eight took 512^3 from 330 to 430 us), writes the quads whose four voxels are sites (distance
// 0: final, most of the field) and lists the others in LDS; its threads then
// search the listed quads one each, so only as many waves as the list needs
// run the search.  Each offset of the disc is one 16-byte load serving a
// quad's four voxels.  The key of the chosen site's offset,
// (dz + 128) << 8 | (dy + 128), orders like (z', y').  IDX is the index type
// (32-bit below 2^32 voxels).
template <typename IDX>
__global__ __launch_bounds__(256) void k_edt1_yz(EnvArgs a, uint32_t* wide, const unsigned long long* b1count)
{
    constexpr int U = 2;
    __shared__ uint16_t list[256 * U];
    __shared__ int wsum[4 * U];
    __shared__ uint32_t stop;
    const IDX nx = (IDX)a.nx, ny = (IDX)a.ny, nz = (IDX)a.nz, plane = nx * ny;
    const IDX nq = plane * nz / 4;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int ntab = c_yz.n;
    // With B1 below 80% of the field the searches would be long and often end
    // beyond the disc: the pass stands down before it reads anything (block 0
    // raises the gate of the separable passes)
    if (*b1count * 5ull < (unsigned long long)(plane * nz) * 4ull) {
        if (blockIdx.x == 0 && tid == 0)
            atomicOr(wide, 1u);
        return;
    }
    bool unsettled = false;
    for (IDX q0 = (IDX)blockIdx.x * (256 * U); q0 < nq; q0 += (IDX)gridDim.x * (256 * U)) {
        uint4 c[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const IDX q = min(q0 + (IDX)(u * 256 + tid), nq - 1);
            c[u] = *reinterpret_cast<const uint4*>(a.win + (int64_t)q * 4);
        }
        // once some block has raised *wide the separable passes recompute the
        // whole field: the rest of this pass is moot (what a block wrote before
        // it stops is overwritten).  Read with the quads, acted on at the list
        // barrier.
        if (tid == 0)
            stop = __hip_atomic_load(wide, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
        uint64_t m[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const IDX q = q0 + (IDX)(u * 256 + tid);
            const bool valid = q < nq;
            const bool sites = ((c[u].x | c[u].y | c[u].z | c[u].w) >> 2) == 0u;
            if (valid && sites)
                *reinterpret_cast<uint4*>(a.w + (int64_t)q * 4) = c[u];
            m[u] = __ballot(valid && !sites);
        }
        // list order: u-major, then wave, then lane
        if (lane == 0) {
#pragma unroll
            for (int u = 0; u < U; ++u)
                wsum[u * 4 + wv] = __popcll(m[u]);
        }
        lds_barrier();
        if (stop)
            break;
        int total = 0, before[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                if (w == wv)
                    before[u] = total;
                total += wsum[u * 4 + w];
            }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if ((m[u] >> lane) & 1ull)
                list[before[u] + __popcll(m[u] & ((1ull << lane) - 1ull))] = (uint16_t)(u * 256 + tid);
        lds_barrier();
#pragma unroll 1
        for (int k = tid; k < total; k += 256) {
            const IDX i = (q0 + (IDX)list[k]) * 4;
            const IDX z = i / plane, y = (i - z * plane) / nx;
            const uint4 cc = *reinterpret_cast<const uint4*>(a.win + (int64_t)i);
            uint32_t bw[4] = {cc.x, cc.y, cc.z, cc.w};
            uint32_t bk[4] = {0x8080u, 0x8080u, 0x8080u, 0x8080u};
            auto limit = [&]() {
                uint32_t l = 0u;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    l = max(l, bw[q] == QAI_WORD_INF ? 0xFFFFu : (bw[q] >> 2));
                return l;
            };
            uint32_t lim = limit();
            // batches of four offsets, uniform over the wave
#pragma unroll 1
            for (int j = 0; j < ntab; j += 4) {
                const bool go = lim >= (c_yz.e[j] >> 16);
                if (__ballot(go) == 0ull)
                    break;
                if (go) {
                    uint4 v[4];
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const uint32_t e = c_yz.e[j + b];
                        const int dz = (int)((e >> 8) & 255u) - 128, dy = (int)(e & 255u) - 128;
                        const int64_t zc = (int64_t)z + dz, yc = (int64_t)y + dy;
                        const bool ok = e != 0xFFFFFFFFu && zc >= 0 && zc < (int64_t)nz && yc >= 0 && yc < (int64_t)ny;
                        // a valid address either way; the value of an offset outside the field is dropped
                        const int64_t o = ok ? (int64_t)i + (int64_t)dz * (int64_t)plane + (int64_t)dy * (int64_t)nx
                                             : (int64_t)i;
                        const uint4 l = *reinterpret_cast<const uint4*>(a.win + o);
                        v[b].x = ok ? l.x : QAI_WORD_INF;
                        v[b].y = ok ? l.y : QAI_WORD_INF;
                        v[b].z = ok ? l.z : QAI_WORD_INF;
                        v[b].w = ok ? l.w : QAI_WORD_INF;
                    }
                    // An absent site (all ones) reads as distance 2^30 - 1, above
                    // every real distance plus d2 (< 3 * 16383^2 + 144), so it
                    // never wins, and any real candidate beats an absent best.
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const uint32_t e = c_yz.e[j + b];
                        const uint32_t d2 = e >> 16, key = e & 0xFFFFu;
                        const uint32_t cw[4] = {v[b].x, v[b].y, v[b].z, v[b].w};
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const uint32_t t = (cw[q] >> 2) + d2, bd = bw[q] >> 2;
                            const bool better = (t < bd) | ((t == bd) & (key < bk[q]));
                            bw[q] = better ? ((t << 2) | (cw[q] & 3u)) : bw[q];
                            bk[q] = better ? key : bk[q];
                        }
                    }
                    lim = limit();
                }
            }
            unsettled |= lim > (uint32_t)YZ_R2;
            *reinterpret_cast<uint4*>(a.w + (int64_t)i) = make_uint4(bw[0], bw[1], bw[2], bw[3]);
        }
        // the list and wsum are rewritten next round; after the last round
        // waves without searches leave at once (their slots go to other blocks)
        if (q0 + (IDX)gridDim.x * (256 * U) < nq)
            lds_barrier();
    }
    if (__ballot(unsettled) != 0ull && lane == 0)
        atomicOr(wide, 1u);
}

static hipError_t launch_edt1_yz(const EnvArgs& a, uint32_t* wide, const unsigned long long* b1count,
                                 bool force_wide, hipStream_t s)
{
    const int64_t n = a.nx * a.ny * a.nz, nq = n / 4;
    const uint32_t grid = grid_cap((uint64_t)((nq + 511) / 512), 1u << 20); // 512 quads per block
    if (n < ((int64_t)1 << 32) && !force_wide)
        return launch_checked(k_edt1_yz<uint32_t>, dim3(grid), dim3(256), 0, s, a, wide, b1count);
    return launch_checked(k_edt1_yz<int64_t>, dim3(grid), dim3(256), 0, s, a, wide, b1count);
}

hipError_t launch_env(int axis, EnvArgs a, const Tuning& t, hipStream_t s)
{
    const int64_t n = axis == 1 ? a.ny : a.nz;
    if (t.env_algo[axis] == 1) {
        int txl = t.env_tx_log2[axis] >= 0 ? t.env_tx_log2[axis] : default_tx_log2(n);
        while (txl > 0 && (n << txl) * 4 > 64 * 1024)
            --txl;
        a.tx_log2 = txl;
        const int64_t nxb = (a.nx + (1 << txl) - 1) >> txl;
        a.ntiles = (uint64_t)(nxb * (axis == 1 ? a.nz : a.ny));
        const uint32_t grid = grid_cap(a.ntiles, 1u << 20);
        const size_t shm = (size_t)(n << txl) * 4;
        const dim3 blk(t.env_threads > 0 ? t.env_threads : 256);
        if (axis == 1)
            return launch_checked(k_env_window<1>, dim3(grid), blk, shm, s, a);
        else
            return launch_checked(k_env_window<2>, dim3(grid), blk, shm, s, a);
    }
    if (t.env_algo[axis] == 2 && n <= 64 * 32)
        return launch_band2(axis, a, t, s);
    if (t.env_algo[axis] == 5) {
        const uint64_t units = (uint64_t)(a.nz * a.ny * ((a.nx + 255) >> 8));
        const dim3 grid(grid_cap(units, 1u << 18)), blk(256);
        return axis == 1 ? launch_checked(k_env_direct<1>, grid, blk, 0, s, a)
                         : launch_checked(k_env_direct<2>, grid, blk, 0, s, a);
    }
    if (t.env_algo[axis] == 4)
        return axis == 1 ? launch_swin_t<1>(a, s) : launch_swin_t<2>(a, s);
    if (t.env_algo[axis] == 3) {
        int hb;
        bool small;
        if (lane2_geometry(axis, a, hb))
            return axis == 1 ? launch_lane2_t<1>(a, hb, s) : launch_lane2_t<2>(a, hb, s);
        if (lane_geometry(axis, a, hb, small)) {
            small = small && !t.force_wide;
            return axis == 1 ? launch_lane_t<1>(a, hb, small, s) : launch_lane_t<2>(a, hb, small, s);
        }
    }
    const int cap = t.stream_cap[axis] <= 16 ? 16 : (t.stream_cap[axis] <= 32 ? 32 : 64);
    const bool fw = t.force_wide != 0;
    if (axis == 1)
        return cap == 16 ? launch_stream_t<1, 16>(a, fw, s)
                         : (cap == 32 ? launch_stream_t<1, 32>(a, fw, s) : launch_stream_t<1, 64>(a, fw, s));
    return cap == 16 ? launch_stream_t<2, 16>(a, fw, s)
                     : (cap == 32 ? launch_stream_t<2, 32>(a, fw, s) : launch_stream_t<2, 64>(a, fw, s));
}

hipError_t launch_interp(const InterpArgs& a, hipStream_t s)
{
    const uint64_t blocks = (uint64_t)((a.n + 255) / 256);
    // gated (only_sparse): a small grid, so that a launch that returns at once
    // costs no dispatch of a block per 256 voxels
    return launch_checked(k_interp, dim3(grid_cap(blocks, a.only_sparse ? 4096u : 1u << 20)), dim3(256), 0, s, a);
}

hipError_t launch_clear(uint32_t* p, int n, hipStream_t s)
{
    return launch_checked(k_clear, dim3((n + 63) / 64), dim3(64), 0, s, p, n);
}

// Which of the three word buffers ends up holding the final words of the
// first EDT (w1) and of the second (w2): the first EDT ping-pongs between
// buffers 0 and 1, the second between the two buffers w1 does not occupy.
void final_buffers(int64_t nz, int64_t ny, int64_t nx, int& w1, int& w2)
{
    (void)nx;
    int cur = 0;
    if (ny > 1)
        cur ^= 1;
    if (nz > 1)
        cur ^= 1;
    w1 = cur;
    const int o0 = w1 == 0 ? 1 : 0;
    const int o1 = w1 == 2 ? 1 : 2;
    int c2 = o0;
    if (ny > 1)
        c2 = (c2 == o0) ? o1 : o0;
    if (nz > 1)
        c2 = (c2 == o0) ? o1 : o0;
    w2 = c2;
}

// Automatic pass algorithm.  The streaming kernels give one wavefront to 64
// columns and walk the whole column, so they need many column tiles to fill
// the GPU; the windowed search is parallel over every voxel but costs the
// distance it searches.  First EDT (short distances): the windowed search
// below 4096 tiles (four waves per SIMD; measured: the y and z passes of a
// sparse-boundary 256^3 field 212 -> 96 us, of 128x128x1024 418 -> 126 us,
// while 512^3 keeps the streaming search, 563 against 1024 us).  Second EDT
// (long distances): the per-lane envelope from 256 tiles on (the windowed
// search took 2.1 ms for the y pass of 100x500x500 and 19 ms at 512^3,
// the envelope 0.14 / 0.67 ms); the windowed search only for passes with very
// few tiles.  The y passes of a 2-D field take the direct per-voxel search
// (the second EDT's only where step E needs it, fused with it, when there
// are no taps): measured on 1800x3600, the first EDT's y pass 100 -> 50 us at
// rel. bound 1e-3, 318 -> 187 us at 1e-2, 43 -> 39 us at 1e-4.
int resolve_algo(int want, bool first_edt, int axis, int64_t nz, int64_t ny, int64_t nx)
{
    if (want >= 0)
        return want;
    if (nz == 1 && axis == 1)
        return 5;
    const int64_t tiles = ((nx + 63) / 64) * (axis == 1 ? nz : ny);
    if (first_edt)
        return tiles < 4096 ? 1 : 4;
    return tiles < 256 ? 1 : 3;
}

static Tuning resolved(const Plan1& p, const Tuning& t_in)
{
    Tuning t = t_in;
    for (int a = 1; a <= 2; ++a) {
        t.edt1_algo[a] = resolve_algo(t_in.edt1_algo[a], true, a, p.nz, p.ny, p.nx);
        t.env_algo[a] = resolve_algo(t_in.env_algo[a], false, a, p.nz, p.ny, p.nx);
    }
    return t;
}

static SeedArgs seed_args(const Plan1& p)
{
    SeedArgs sa = {};
    sa.xq = p.xq;
    sa.nx = p.nx;
    sa.ny = p.ny;
    sa.nz = p.nz;
    sa.two_eb = 2.0f * p.eb;
    sa.inv2eb = 1.0f / sa.two_eb;
    sa.status = p.status;
    sa.tq = p.taps.q;
    sa.tb1 = p.taps.b1;
    sa.tsb = p.taps.sb;
    sa.ts = p.taps.s;
    sa.td1 = p.taps.d1sq;
    sa.tb2 = p.taps.b2;
    return sa;
}

// A 3-D field with both passes of the first EDT on automatic takes them as
// one search over (y, z) (k_edt1_yz); its seed pass (k_seed_lane) then
// estimates the B1 count, which the later passes read on the device.
// The first seed pass estimates B1 on 3-D fields whenever it is the
// register-resident kernel (the fused first-EDT search and the choice between
// the needed-voxel search and a whole z pass read the estimate).
static bool b1_estimated(const Plan1& p, const Tuning& t)
{
    return p.nz > 1 && p.ny > 1 && t.seed_ty == 0 && p.nx <= kSeedLaneMaxX;
}

static bool fused_edt1(const Plan1& p, const Tuning& t, const Tuning& t_in)
{
    return p.nz > 1 && p.ny > 1 && p.nx % 4 == 0 && p.nx <= 512 && t.seed_ty == 0 && t_in.edt1_algo[1] < 0 &&
           t_in.edt1_algo[2] < 0;
}

// Steps A and B (and the status words): afterwards the first EDT's final
// words lie in word buffer *w1 (0, 1 or 2).
hipError_t run_part1(Plan1& p, const Tuning& t_in, hipStream_t s, int* w1)
{
    const Tuning t = resolved(p, t_in);
    uint32_t* buf[3] = {p.bufA, p.bufB, p.bufC};
    prof_begin("clear", s);
    QAI_TRY(launch_clear(p.status, QAI_HEADER_WORDS, s));
    prof_end(s);

    SeedArgs sa = seed_args(p);

    // step A + x pass of step B; a 3-D field with both passes of the first
    // EDT on automatic takes them as one search over (y, z) (k_edt1_yz), the
    // separable passes gated behind it; the final words land in buffer 0
    // either way
    const bool yz = fused_edt1(p, t, t_in);
    unsigned long long* const b1count = (unsigned long long*)(p.status + QAI_B1_WORD);
    sa.b1count = (yz || b1_estimated(p, t)) ? b1count : nullptr;
    int cur = yz ? 1 : 0;
    sa.wout = buf[cur];
    if (p.coded && coded_seed_supported(p.nx) && t.seed_ty == 0) {
        // decode inside the seed pass, which also writes x' into out; the
        // later stages then take out as their x' (in place)
        sa.cbase = p.coded->base;
        sa.cmeta = p.coded->meta;
        sa.cpay = p.coded->payload;
        sa.cpay_bytes = (uint32_t)(p.coded->payload_words * 4);
        sa.segs_row = (p.nx + 31) / 32;
        sa.xout = p.out;
        prof_begin("seed1_xscan", s);
        QAI_TRY(launch_seed_coded(sa, p.nz > 1 ? (t.seed_tz > 0 ? t.seed_tz : 16) : 1, s));
        prof_end(s);
        p.xq = p.out;
    } else {
        if (p.coded) {
            // other line shapes: decode x' into out first, then the plain pass in place
            prof_begin("decode", s);
            QAI_TRY(launch_decode(*p.coded, p.nz, p.ny, p.nx, 2.0f * p.eb, p.out, s));
            prof_end(s);
            p.xq = p.out;
            sa.xq = p.out;
        }
        prof_begin("seed1_xscan", s);
        QAI_TRY(launch_seed(0, sa, s, t.seed_ty, t.seed_tz));
        prof_end(s);
    }

    EnvArgs ea = {};
    ea.nx = p.nx;
    ea.ny = p.ny;
    ea.nz = p.nz;
    Tuning t1 = t; // the first EDT: dense boundaries, short owner distances
    for (int i = 0; i < 3; ++i) {
        t1.stream_cap[i] = t.edt1_cap[i];
        t1.env_algo[i] = t.edt1_algo[i];
    }
    if (yz) {
        uint32_t* wide = p.status + QAI_WIDE_WORD;
        ea.win = buf[1];
        ea.w = buf[0];
        prof_begin("edt1_yz", s);
        QAI_TRY(launch_edt1_yz(ea, wide, b1count, t.force_wide != 0, s));
        prof_end(s);
        // the fallback, gated: the separable passes with the automatic choice
        // for each axis (both candidate kernels read the gate)
        Tuning tf = t1;
        tf.env_algo[1] = resolve_algo(-1, true, 1, p.nz, p.ny, p.nx);
        tf.env_algo[2] = resolve_algo(-1, true, 2, p.nz, p.ny, p.nx);
        ea.gate = wide;
        prof_begin("edt1_fallback", s);
        ea.win = buf[1];
        ea.w = buf[2];
        QAI_TRY(launch_env(1, ea, tf, s));
        ea.win = buf[2];
        ea.w = buf[0];
        QAI_TRY(launch_env(2, ea, tf, s));
        prof_end(s);
        ea.gate = nullptr;
        cur = 0;
    } else if (p.ny > 1) {
        ea.win = buf[cur];
        ea.w = buf[cur ^ 1];
        prof_begin("edt1_y", s);
        QAI_TRY(launch_env(1, ea, t1, s));
        prof_end(s);
        cur ^= 1;
    }
    if (p.nz > 1 && !yz) {
        ea.win = buf[cur];
        ea.w = buf[cur ^ 1];
        prof_begin("edt1_z", s);
        QAI_TRY(launch_env(2, ea, t1, s));
        prof_end(s);
        cur ^= 1;
    }
    *w1 = cur;
    return hipSuccess;
}

// Steps C, D and E on the first EDT's words in buffer w1.
hipError_t run_part2(Plan1& p, const Tuning& t_in, hipStream_t s, int w1)
{
    const Tuning t = resolved(p, t_in);
    uint32_t* buf[3] = {p.bufA, p.bufB, p.bufC};
    SeedArgs sa = seed_args(p);
    EnvArgs ea = {};
    ea.nx = p.nx;
    ea.ny = p.ny;
    ea.nz = p.nz;

    // step C + x pass of step D
    const int o0 = w1 == 0 ? 1 : 0, o1 = w1 == 2 ? 1 : 2;
    int c2 = o0;
    sa.w1 = buf[w1];
    sa.wout = buf[c2];
    prof_begin("seed2_xscan", s);
    sa.b1count = nullptr;
    QAI_TRY(launch_seed(1, sa, s, t.seed_ty, t.seed_tz));
    prof_end(s);

    // remaining passes of step D; without taps, a 3-D field's last pass runs
    // only where step E needs it (the needed-voxel search).  When the
    // per-lane envelope runs the y pass ahead of it, the y pass hands its
    // result over in the layout blocked_layout picks from the B1 estimate
    // (blocked where there is no estimate)
    const qai_taps& tp = p.taps;
    const bool any_tap = tp.q || tp.b1 || tp.sb || tp.s || tp.d1sq || tp.b2 || tp.d2sq || tp.w;
    const bool aligned = (((uintptr_t)buf[w1] | (uintptr_t)p.xq | (uintptr_t)p.out) & 15u) == 0;
    const bool search = p.nz > 1 && !any_tap && t_in.env_algo[2] < 0 && p.flags && aligned;
    // a 2-D field's last pass (y) only where step E needs it, fused with step
    // E, when the y pass is on automatic or the direct search
    const bool search2d = p.nz == 1 && p.ny > 1 && !any_tap && (t_in.env_algo[1] < 0 || t_in.env_algo[1] == 5);
    // the streaming phase of step E needs only the x-pass words: with a side
    // stream it runs there while the y pass (issue-bound, LDS-limited to a
    // few waves per SIMD) runs here; the search phase joins after both
    const bool overlap = search && p.ny > 1 && p.aux;
    if (overlap) {
        const int w2b = o0; // the search phase's distance words: the x-pass buffer (see nx2 below)
        ZsArgs zp = {buf[w1], nullptr, buf[w2b], p.xq, p.out, p.flags, p.nx, p.ny, p.nz, p.eta * p.eb, p.power, false,
                     nullptr, nullptr, buf[c2]};
        QAI_TRY(hipEventRecord(p.aux->fork, s));
        QAI_TRY(hipStreamWaitEvent(p.aux->s, p.aux->fork, 0));
        prof_begin("edt2_z_stream", p.aux->s);
        QAI_TRY(launch_interp_stream(zp, t.force_wide != 0, true, p.aux->s));
        prof_end(p.aux->s);
        QAI_TRY(hipEventRecord(p.aux->join, p.aux->s));
    }
    if (search2d) {
        ZsArgs zd = {buf[w1], nullptr, buf[o1], p.xq, p.out, nullptr, p.nx, p.ny, p.nz, p.eta * p.eb, p.power, false,
                     nullptr, nullptr, buf[c2]};
        prof_begin("edt2_y_interp", s);
        QAI_TRY(launch_interp_dir(zd, s));
        prof_end(s);
        p.w1_final = buf[w1];
        p.w2_final = buf[o1];
        return hipSuccess;
    }
    bool blk = false;
    const unsigned long long* b1est = nullptr;
    uint32_t* ovf = nullptr;
    if (p.ny > 1) {
        const int nx2 = (c2 == o0) ? o1 : o0;
        ea.win = buf[c2];
        ea.w = buf[nx2];
        int hb = 0;
        const bool lane = t.env_algo[1] == 3 && lane2_geometry(1, ea, hb);
        blk = search && lane;
        if (blk && b1_estimated(p, t))
            b1est = (const unsigned long long*)(p.status + QAI_B1_WORD);
        // columns whose envelope outgrows the per-lane ring (sparse B2 over
        // long x-lines) hand the pass to the banded pass, gated on a header word
        // (ahead of a whole z pass too: the ring size and the hand-off then
        // serve it as they serve the search)
        if (lane && p.ny <= 64 * 32)
            ovf = p.status + QAI_OVF_WORD;
        prof_begin("edt2_y", s);
        if (lane)
            QAI_TRY(launch_lane2_y(ea, hb, b1est, ovf, !blk, s));
        else
            QAI_TRY(launch_env(1, ea, t, s));
        if (ovf) {
            EnvArgs eg = ea;
            eg.gate = ovf;
            QAI_TRY(launch_band2(1, eg, t, s));
        }
        prof_end(s);
        c2 = nx2;
    }
    if (search) {
        // last pass of step D only at needed voxels, fused with step E
        const int nx2 = (c2 == o0) ? o1 : o0;
        ZsArgs za = {buf[w1], buf[c2], buf[nx2], p.xq, p.out, p.flags, p.nx, p.ny, p.nz, p.eta * p.eb, p.power, blk,
                     b1est, ovf, nullptr, nullptr};
        if (overlap) {
            if (nx2 != o0)
                return hipErrorInvalidValue; // the streaming phase relied on w2 being the x-pass buffer
            QAI_TRY(hipStreamWaitEvent(s, p.aux->join, 0));
            // with the B1 estimate at hand, the whole z pass and step E at the
            // voxels the search would take go to the side stream beside the
            // search, each gated on sparse_b1
            EnvArgs ez = ea;
            ez.win = buf[c2];
            ez.w = buf[nx2];
            ez.gate = nullptr;
            int hbz = 0;
            const unsigned long long* b1all = (const unsigned long long*)(p.status + QAI_B1_WORD);
            // (passes of at most 2048 column tiles: on larger ones the gated
            // envelope's blocks, which hold its LDS ring, wait beside the
            // search's and delay it even when they return at once: 512^3
            // 1.600 -> 1.614 ms)
            const bool dual = b1_estimated(p, t) && p.nz <= 64 * 32 && ((p.nx + 63) / 64) * p.ny <= 2048 &&
                              lane2_geometry(2, ez, hbz);
            if (dual) {
                // (no banded pass behind it: its gated launch would wait for
                // LDS behind the search's blocks; overflowing columns take the
                // envelope kernel's own exact outward search)
                QAI_TRY(hipEventRecord(p.aux->fork, s));
                QAI_TRY(hipStreamWaitEvent(p.aux->s, p.aux->fork, 0));
                prof_begin("edt2_z_sparse", p.aux->s);
                QAI_TRY(launch_lane2_z(ez, hbz, nullptr, b1all, p.aux->s));
                InterpArgs ia = {buf[w1], buf[nx2], p.xq, p.out, p.nx * p.ny * p.nz, p.eta * p.eb, p.power, nullptr,
                                 nullptr, b1all};
                QAI_TRY(launch_interp(ia, p.aux->s));
                prof_end(p.aux->s);
                QAI_TRY(hipEventRecord(p.aux->join, p.aux->s));
                za.skip_sparse = b1all;
            }
            prof_begin("edt2_z_search", s);
            QAI_TRY(launch_interp_far(za, t.force_wide != 0, s));
            prof_end(s);
            if (dual)
                QAI_TRY(hipStreamWaitEvent(s, p.aux->join, 0));
        } else {
            prof_begin("edt2_z_interp", s);
            QAI_TRY(launch_interp_stream(za, t.force_wide != 0, false, s));
            QAI_TRY(launch_interp_far(za, t.force_wide != 0, s));
            prof_end(s);
        }
        p.w1_final = buf[w1];
        p.w2_final = buf[nx2];
        return hipSuccess;
    }
    if (p.nz > 1) {
        const int nx2 = (c2 == o0) ? o1 : o0;
        ea.win = buf[c2];
        ea.w = buf[nx2];
        ea.gate = nullptr;
        int hb = 0;
        prof_begin("edt2_z", s);
        if (t.env_algo[2] == 3 && p.nz <= 64 * 32 && lane2_geometry(2, ea, hb)) {
            // per-lane envelope with the banded pass behind it for columns
            // that outgrow the ring
            uint32_t* ovfz = p.status + QAI_OVFZ_WORD;
            QAI_TRY(launch_lane2_z(ea, hb, ovfz, nullptr, s));
            EnvArgs eg = ea;
            eg.gate = ovfz;
            QAI_TRY(launch_band2(2, eg, t, s));
        } else {
            QAI_TRY(launch_env(2, ea, t, s));
        }
        prof_end(s);
        c2 = nx2;
    }

    // step E
    InterpArgs ia = {buf[w1], buf[c2], p.xq, p.out, p.nx * p.ny * p.nz, p.eta * p.eb, p.power, p.taps.d2sq, p.taps.w};
    prof_begin("interp", s);
    QAI_TRY(launch_interp(ia, s));
    prof_end(s);
    p.w1_final = buf[w1];
    p.w2_final = buf[c2];
    return hipSuccess;
}

static std::mutex g_aux_mu;
static Aux g_aux[64];

hipError_t aux_for(int dev, Aux*& out)
{
    out = nullptr;
    if (dev < 0 || dev >= 64)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_aux_mu);
    Aux& x = g_aux[dev];
    if (!x.s) {
        hipStream_t st = nullptr;
        hipEvent_t f = nullptr, j = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&f, hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&j, hipEventDisableTiming);
        if (e != hipSuccess) {
            if (j) (void)hipEventDestroy(j);
            if (f) (void)hipEventDestroy(f);
            if (st) (void)hipStreamDestroy(st);
            return e;
        }
        x.fork = f;
        x.join = j;
        x.s = st;
    }
    out = &x;
    return hipSuccess;
}

bool stream_capturing(hipStream_t s)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &st) != hipSuccess || st != hipStreamCaptureStatusNone;
}

hipError_t run_plain(Plan1& p, const Tuning& t, hipStream_t s)
{
    int w1 = 0;
    QAI_TRY(run_part1(p, t, s, &w1));
    return run_part2(p, t, s, w1);
}

} // namespace qai
