// qai_plain.hip -- kernels of the plain QAI post-pass for gfx950.
//
// Stage map (Algorithm 4 of the paper):
//   k_seed_xscan<0>  step A (Algorithm 2) fused with the x pass of step B:
//                    x' -> q -> B1 and S_B by a 6-neighbour stencil, then
//                    each voxel's nearest B1 voxel on its x-line.
//   k_env<y|z>       remaining passes of step B: exact 1-D lower-envelope
//                    minimisation of g(j) + (i - j)^2 along y, then z
//                    (Algorithm 1's result, sign payload carried along).
//   k_seed_xscan<1>  step C (Algorithm 3): propagated S read from the final
//                    words, B2 by a 6-neighbour stencil, then the x pass of
//                    step D.
//   k_env<y|z>       remaining passes of step D; the last one ends with
//                    step E (interpolation and compensation) in registers.
// All kernels are memory bound: no dense contraction exists on this path.
#include "qai_device.h"
#include "qai_kernels.h"

namespace qai {

// ------------------------------------------------------------------ seeds
// One wave per x-line.  Forward sweep over 64-voxel chunks: stencil, site
// flags by ballot, per-chunk masks and the last site before each chunk kept
// in LDS.  Backward sweep: nearest site to the left (highest set bit at or
// below the lane, else the carried one) and to the right; the left one wins
// ties (lower x, as Algorithm 1's strict query comparison).
template <int MODE>
__global__ __launch_bounds__(256) void k_seed_xscan(SeedArgs a)
{
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

    for (uint64_t t = blockIdx.x; t < a.ngroups; t += gridDim.x) {
        const uint64_t grp = xcd_remap(t, a.ngroups);
        const int64_t line = (int64_t)grp * a.waves + wave;
        if (line >= lines)
            continue;
        const int64_t y = line % ny, z = line / ny;
        const int64_t base = line * nx;
        const bool line_in = (ny == 1 || (y >= 1 && y <= ny - 2)) && (nz == 1 || (z >= 1 && z <= nz - 2));
        bool bad = false;

        int last = -1;   // last site before the current chunk
        int kprev = 0;   // key at x = 64c - 1
        for (int c = 0; c < nch; ++c) {
            const int64_t x = (int64_t)c * 64 + lane;
            const bool valid = x < nx;
            int kc = 0;
            uint32_t wc = QAI_WORD_INF;
            if (valid) {
                if (MODE == 0) {
                    kc = recover_q(a.xq[base + x], a.inv2eb, a.two_eb, bad);
                } else {
                    wc = a.w1[base + x];
                    kc = word_sign(wc);
                }
            }
            int km = __shfl_up(kc, 1);
            int kp = __shfl_down(kc, 1);
            if (lane == 0)
                km = kprev;
            if (lane == 63 && x + 1 < nx) {
                if (MODE == 0)
                    kp = recover_q(a.xq[base + x + 1], a.inv2eb, a.two_eb, bad);
                else
                    kp = word_sign(a.w1[base + x + 1]);
            }
            kprev = __shfl(kc, 63);

            const bool x_in = (nx == 1) || (x >= 1 && x <= nx - 2);
            bool site = false;
            int sgn = 0;
            if (valid && line_in && x_in) {
                if (MODE == 0) {
                    // Algorithm 2: boundary if some 6-neighbour index differs; sign of the
                    // first differing neighbour (+x, -x, +y, -y, +z, -z); discarded where an
                    // absolute central difference reaches 1 (|q+ - q-| >= 2).
                    int first = 0;
                    bool steep = false;
                    if (nx > 1) {
                        first = (kp != kc) ? kp - kc : ((km != kc) ? km - kc : 0);
                        steep = abs(kp - km) >= 2;
                    }
                    if (ny > 1) {
                        int a1 = recover_q(a.xq[base + x + nx], a.inv2eb, a.two_eb, bad);
                        int a0 = recover_q(a.xq[base + x - nx], a.inv2eb, a.two_eb, bad);
                        if (first == 0)
                            first = (a1 != kc) ? a1 - kc : ((a0 != kc) ? a0 - kc : 0);
                        steep = steep || abs(a1 - a0) >= 2;
                    }
                    if (nz > 1) {
                        int a1 = recover_q(a.xq[base + x + plane], a.inv2eb, a.two_eb, bad);
                        int a0 = recover_q(a.xq[base + x - plane], a.inv2eb, a.two_eb, bad);
                        if (first == 0)
                            first = (a1 != kc) ? a1 - kc : ((a0 != kc) ? a0 - kc : 0);
                        steep = steep || abs(a1 - a0) >= 2;
                    }
                    if (first != 0) {
                        site = true;
                        sgn = steep ? 0 : (first > 0 ? 1 : -1);
                    }
                } else {
                    // Algorithm 3's GetBoundary(S): interior voxels outside B1 whose
                    // propagated sign differs from a 6-neighbour's.
                    const bool on_b1 = (wc != QAI_WORD_INF) && (word_d2(wc) == 0u);
                    if (!on_b1) {
                        bool diff = false;
                        if (nx > 1)
                            diff = (kp != kc) || (km != kc);
                        if (ny > 1 && !diff)
                            diff = (word_sign(a.w1[base + x + nx]) != kc) || (word_sign(a.w1[base + x - nx]) != kc);
                        if (nz > 1 && !diff)
                            diff = (word_sign(a.w1[base + x + plane]) != kc) ||
                                   (word_sign(a.w1[base + x - plane]) != kc);
                        site = diff;
                    }
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
                    if (a.ts) a.ts[i] = (int8_t)kc;
                    if (a.td1) a.td1[i] = (wc == QAI_WORD_INF) ? -1 : (int32_t)word_d2(wc);
                    if (a.tb2) a.tb2[i] = site ? 1 : 0;
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

__global__ __launch_bounds__(256) void k_interp(InterpArgs a)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * blockDim.x)
        interp_store(i, a.w2[i], a.w1, a.xq, a.out, a.eta_eb, a.power, a.td2, a.tw);
}

// --------------------------------------------------------- envelope pass
// Exact 1-D minimisation D(i) = min_j g(j) + (i - j)^2 along the pass axis
// for a tile of adjacent x-columns, whole lines staged in LDS.  Candidates
// are visited outward from i (offset d = 1, 2, ...); the search stops once
// d^2 exceeds the best value found, since every farther candidate is at
// least d^2.  At equal value the lower coordinate wins (left candidates win
// ties, right ones need to be strictly better), the choice Algorithm 1's
// strict comparisons make.
template <int AXIS, bool EPI>
__global__ __launch_bounds__(256) void k_env_window(EnvArgs a)
{
    extern __shared__ __align__(16) uint32_t tile[];
    const int txl = a.tx_log2;
    const int Tx = 1 << txl;
    const int64_t n = (AXIS == 1) ? a.ny : a.nz;
    const int64_t stride = (AXIS == 1) ? a.nx : a.nx * a.ny;
    const int64_t nxb = (a.nx + Tx - 1) >> txl;
    const int total = (int)(n << txl);

    for (uint64_t t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
        const uint64_t tl = xcd_remap(t, a.ntiles);
        const int64_t xb = (int64_t)(tl % (uint64_t)nxb), o = (int64_t)(tl / (uint64_t)nxb);
        const int64_t x0 = xb << txl;
        const int64_t base = (AXIS == 1) ? o * a.nx * a.ny + x0 : o * a.nx + x0;
        __syncthreads();
        for (int i = threadIdx.x; i < total; i += blockDim.x) {
            const int r = i >> txl, c = i & (Tx - 1);
            tile[i] = (x0 + c < a.nx) ? a.w[base + (int64_t)r * stride + c] : QAI_WORD_INF;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < total; i += blockDim.x) {
            const int r = i >> txl, c = i & (Tx - 1);
            if (x0 + c >= a.nx)
                continue;
            uint32_t best = tile[i];
            for (int d = 1; d < n; ++d) {
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
            const int64_t gi = base + (int64_t)r * stride + c;
            if (a.write_words)
                a.w[gi] = best;
            if (EPI)
                interp_store(gi, best, a.w1, a.xq, a.out, a.eta_eb, a.power, a.td2, a.tw);
        }
    }
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
    t.env_tx_log2[0] = t.env_tx_log2[1] = t.env_tx_log2[2] = -1;
    t.env_threads = 256;
}

hipError_t launch_seed(int mode, const SeedArgs& in, hipStream_t s)
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
        hipLaunchKernelGGL(k_seed_xscan<0>, dim3(grid), dim3(64 * waves), shm, s, a);
    else
        hipLaunchKernelGGL(k_seed_xscan<1>, dim3(grid), dim3(64 * waves), shm, s, a);
    return hipGetLastError();
}

static int default_tx_log2(int64_t n)
{
    // keep the staged tile within 32 KB: several workgroups share a CU
    int l = 4;
    while (l > 0 && (n << l) * 4 > 32 * 1024)
        --l;
    return l;
}

hipError_t launch_env(int axis, bool epi, EnvArgs a, const Tuning& t, hipStream_t s)
{
    const int64_t n = axis == 1 ? a.ny : a.nz;
    int txl = t.env_tx_log2[axis] >= 0 ? t.env_tx_log2[axis] : default_tx_log2(n);
    while (txl > 0 && (n << txl) * 4 > 64 * 1024)
        --txl;
    a.tx_log2 = txl;
    const int64_t nxb = (a.nx + (1 << txl) - 1) >> txl;
    a.ntiles = (uint64_t)(nxb * (axis == 1 ? a.nz : a.ny));
    const uint32_t grid = grid_cap(a.ntiles, 1u << 20);
    const size_t shm = (size_t)(n << txl) * 4;
    const dim3 blk(t.env_threads > 0 ? t.env_threads : 256);
    if (axis == 1) {
        if (epi) hipLaunchKernelGGL((k_env_window<1, true>), dim3(grid), blk, shm, s, a);
        else hipLaunchKernelGGL((k_env_window<1, false>), dim3(grid), blk, shm, s, a);
    } else {
        if (epi) hipLaunchKernelGGL((k_env_window<2, true>), dim3(grid), blk, shm, s, a);
        else hipLaunchKernelGGL((k_env_window<2, false>), dim3(grid), blk, shm, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_interp(const InterpArgs& a, hipStream_t s)
{
    const uint64_t blocks = (uint64_t)((a.n + 255) / 256);
    hipLaunchKernelGGL(k_interp, dim3(grid_cap(blocks, 1u << 20)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_clear(uint32_t* p, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_clear, dim3((n + 63) / 64), dim3(64), 0, s, p, n);
    return hipGetLastError();
}

#define QAI_TRY(expr)                   \
    do {                                \
        hipError_t e_ = (expr);         \
        if (e_ != hipSuccess)           \
            return e_;                  \
    } while (0)

hipError_t run_plain(const Plan1& p, const Tuning& t, hipStream_t s)
{
    const float eta_eb = p.eta * p.eb;
    prof_begin("clear", s);
    QAI_TRY(launch_clear(p.status, 1, s));
    prof_end(s);

    SeedArgs sa = {};
    sa.xq = p.xq;
    sa.w1 = p.w1;
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

    // step A + x pass of step B
    sa.wout = p.w1;
    prof_begin("seed1_xscan", s);
    QAI_TRY(launch_seed(0, sa, s));
    prof_end(s);

    EnvArgs ea = {};
    ea.nx = p.nx;
    ea.ny = p.ny;
    ea.nz = p.nz;
    ea.write_words = true;
    ea.w = p.w1;
    if (p.ny > 1) {
        prof_begin("edt1_y", s);
        QAI_TRY(launch_env(1, false, ea, t, s));
        prof_end(s);
    }
    if (p.nz > 1) {
        prof_begin("edt1_z", s);
        QAI_TRY(launch_env(2, false, ea, t, s));
        prof_end(s);
    }

    // step C + x pass of step D
    sa.wout = p.w2;
    prof_begin("seed2_xscan", s);
    QAI_TRY(launch_seed(1, sa, s));
    prof_end(s);

    // remaining passes of step D; the last one carries step E
    ea.w = p.w2;
    ea.w1 = p.w1;
    ea.xq = p.xq;
    ea.out = p.out;
    ea.eta_eb = eta_eb;
    ea.power = p.power;
    ea.td2 = p.taps.d2sq;
    ea.tw = p.taps.w;
    if (p.nz > 1) {
        if (p.ny > 1) {
            prof_begin("edt2_y", s);
            QAI_TRY(launch_env(1, false, ea, t, s));
            prof_end(s);
        }
        ea.write_words = p.keep_w2;
        prof_begin("edt2_z_interp", s);
        QAI_TRY(launch_env(2, true, ea, t, s));
        prof_end(s);
    } else if (p.ny > 1) {
        ea.write_words = p.keep_w2;
        prof_begin("edt2_y_interp", s);
        QAI_TRY(launch_env(1, true, ea, t, s));
        prof_end(s);
    } else {
        InterpArgs ia = {p.w1, p.w2, p.xq, p.out, p.nx, eta_eb, p.power, p.taps.d2sq, p.taps.w};
        prof_begin("interp", s);
        QAI_TRY(launch_interp(ia, s));
        prof_end(s);
    }
    return hipSuccess;
}

} // namespace qai
