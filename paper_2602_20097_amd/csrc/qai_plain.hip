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

// Banded exact lower envelope (the result of Algorithm 1 on every line of a
// tile, computed with all threads of the workgroup).
//
// A tile is Tx adjacent x-columns by the whole line along the pass axis,
// staged in LDS.  Each line is cut into bands of m positions, one thread per
// (column, band):
//   1. every thread builds the lower envelope of the sites of its band with
//      Algorithm 1's stack (RemoveEDT), kept as a doubly linked list in LDS;
//   2. log2(bands) levels merge neighbouring envelopes pairwise: the left
//      list's tail and the right list's head are trimmed with the same
//      predicate until both junction triples are kept;
//   3. every thread walks to the site owning its first position (values
//      along the list are unimodal there) and advances monotonically through
//      its band, keeping the lower site on equal values.
// Removed sites are strictly dominated everywhere, so the survivors and the
// chosen sites are exactly those of Algorithm 1's stack and query.
struct BandLds {
    uint32_t* G;    // [n][Tx] packed words of the sites (QAI_WORD_INF: none)
    int16_t* PREV;  // [n][Tx] list links; -2 marks a removed site
    int16_t* NEXT;  // [n][Tx]
    int16_t* HEAD;  // [B][Tx] first / last element of a (merged) band list
    int16_t* TAIL;
    int16_t* FIRST; // [B][Tx] first / last surviving site inside each band
    int16_t* LAST;
    unsigned long long* MASK; // [Tx] bands holding a survivor
};

__device__ __forceinline__ size_t band_lds_bytes(int n, int B, int Tx)
{
    return (size_t)n * Tx * 8 + (size_t)B * Tx * 8 + (size_t)Tx * 8 + 64;
}

__device__ __forceinline__ BandLds band_lds(unsigned char* smem, int n, int B, int Tx)
{
    BandLds L;
    unsigned long long* mask = (unsigned long long*)smem;
    L.MASK = mask;
    L.G = (uint32_t*)(smem + (size_t)Tx * 8);
    L.PREV = (int16_t*)(L.G + (size_t)n * Tx);
    L.NEXT = L.PREV + (size_t)n * Tx;
    L.HEAD = L.NEXT + (size_t)n * Tx;
    L.TAIL = L.HEAD + (size_t)B * Tx;
    L.FIRST = L.TAIL + (size_t)B * Tx;
    L.LAST = L.FIRST + (size_t)B * Tx;
    return L;
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

template <int AXIS, bool EPI>
__global__ __launch_bounds__(1024) void k_env_band(EnvArgs a, int m, int B)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int txl = a.tx_log2;
    const int Tx = 1 << txl;
    const int n = (int)((AXIS == 1) ? a.ny : a.nz);
    const int64_t stride = (AXIS == 1) ? a.nx : a.nx * a.ny;
    const int64_t nxb = (a.nx + Tx - 1) >> txl;
    const int total = n << txl;
    BandLds L = band_lds(smem, n, B, Tx);
    const int tid = threadIdx.x;
    const int c = tid & (Tx - 1);
    const int b = tid >> txl;
    const bool active = b < B;
    const int p0 = b * m;
    const int p1 = min(n, p0 + m);

    for (uint64_t t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
        const uint64_t tl = xcd_remap(t, a.ntiles);
        const int64_t xb = (int64_t)(tl % (uint64_t)nxb), o = (int64_t)(tl / (uint64_t)nxb);
        const int64_t x0 = xb << txl;
        const int64_t base = (AXIS == 1) ? o * a.nx * a.ny + x0 : o * a.nx + x0;
        __syncthreads();
        for (int i = tid; i < total; i += blockDim.x) {
            const int r = i >> txl, cc = i & (Tx - 1);
            L.G[i] = (x0 + cc < a.nx) ? a.w[base + (int64_t)r * stride + cc] : QAI_WORD_INF;
        }
        if (tid < Tx)
            L.MASK[tid] = 0ull;
        __syncthreads();

        // 1. envelope of each band
        if (active) {
            int top = -1, second = -1, head = -1;
            uint32_t gtop = 0, gsec = 0;
            for (int p = p0; p < p1; ++p) {
                const uint32_t w = L.G[(p << txl) + c];
                if (w == QAI_WORD_INF)
                    continue;
                const uint32_t g = w >> 2;
                for (int it = 0; it < m && second >= 0 && remove_mid(gsec, gtop, g, second, top, p); ++it) {
                    L.PREV[(top << txl) + c] = -2;
                    top = second;
                    gtop = gsec;
                    second = L.PREV[(second << txl) + c];
                    gsec = second >= 0 ? (L.G[(second << txl) + c] >> 2) : 0u;
                }
                L.PREV[(p << txl) + c] = (int16_t)top;
                if (top >= 0)
                    L.NEXT[(top << txl) + c] = (int16_t)p;
                else
                    head = p;
                second = top;
                gsec = gtop;
                top = p;
                gtop = g;
            }
            if (top >= 0)
                L.NEXT[(top << txl) + c] = -1;
            L.HEAD[(b << txl) + c] = (int16_t)head;
            L.TAIL[(b << txl) + c] = (int16_t)top;
        }
        __syncthreads();

        // 2. pairwise merges
        for (int span = 1; span < B; span <<= 1) {
            if (active && (b & (2 * span - 1)) == 0 && b + span < B) {
                const int r = b + span;
                const int tl_ = L.TAIL[(b << txl) + c];
                const int tr = L.TAIL[(r << txl) + c];
                if (tl_ < 0) {
                    L.HEAD[(b << txl) + c] = L.HEAD[(r << txl) + c];
                    L.TAIL[(b << txl) + c] = (int16_t)tr;
                } else if (tr >= 0) {
                    int t1 = tl_, t0 = L.PREV[(t1 << txl) + c];
                    int h1 = L.HEAD[(r << txl) + c], h2 = L.NEXT[(h1 << txl) + c];
                    uint32_t g_t1 = L.G[(t1 << txl) + c] >> 2, g_h1 = L.G[(h1 << txl) + c] >> 2;
                    uint32_t g_t0 = t0 >= 0 ? (L.G[(t0 << txl) + c] >> 2) : 0u;
                    uint32_t g_h2 = h2 >= 0 ? (L.G[(h2 << txl) + c] >> 2) : 0u;
                    for (int it = 0; it < n; ++it) {
                        if (t0 >= 0 && remove_mid(g_t0, g_t1, g_h1, t0, t1, h1)) {
                            L.PREV[(t1 << txl) + c] = -2;
                            t1 = t0;
                            g_t1 = g_t0;
                            t0 = L.PREV[(t0 << txl) + c];
                            g_t0 = t0 >= 0 ? (L.G[(t0 << txl) + c] >> 2) : 0u;
                            continue;
                        }
                        if (h2 >= 0 && remove_mid(g_t1, g_h1, g_h2, t1, h1, h2)) {
                            L.PREV[(h1 << txl) + c] = -2;
                            h1 = h2;
                            g_h1 = g_h2;
                            h2 = L.NEXT[(h2 << txl) + c];
                            g_h2 = h2 >= 0 ? (L.G[(h2 << txl) + c] >> 2) : 0u;
                            continue;
                        }
                        break;
                    }
                    L.NEXT[(t1 << txl) + c] = (int16_t)h1;
                    L.PREV[(h1 << txl) + c] = (int16_t)t1;
                    L.TAIL[(b << txl) + c] = (int16_t)tr;
                }
            }
            __syncthreads();
        }

        // survivors inside each band
        if (active) {
            int first = -1, last = -1;
            for (int p = p0; p < p1; ++p) {
                const int i = (p << txl) + c;
                if (L.G[i] != QAI_WORD_INF && L.PREV[i] != -2) {
                    if (first < 0)
                        first = p;
                    last = p;
                }
            }
            L.FIRST[(b << txl) + c] = (int16_t)first;
            L.LAST[(b << txl) + c] = (int16_t)last;
            if (first >= 0)
                atomicOr(&L.MASK[c], 1ull << b);
        }
        __syncthreads();

        // 3. query
        if (active && x0 + c < a.nx) {
            const unsigned long long mk = L.MASK[c];
            int s = L.FIRST[(b << txl) + c];
            if (s < 0 && mk) {
                const unsigned long long below = (b == 0) ? 0ull : (mk & ((1ull << b) - 1ull));
                if (below)
                    s = L.LAST[((63 - __clzll(below)) << txl) + c];
                else
                    s = L.FIRST[((__ffsll(mk) - 1) << txl) + c];
            }
            if (s < 0) {
                for (int p = p0; p < p1; ++p) {
                    const int64_t gi = base + (int64_t)p * stride + c;
                    if (a.write_words)
                        a.w[gi] = QAI_WORD_INF;
                    if (EPI)
                        interp_store(gi, QAI_WORD_INF, a.w1, a.xq, a.out, a.eta_eb, a.power, a.td2, a.tw);
                }
            } else {
                int o = s;
                uint32_t wo = L.G[(o << txl) + c];
                for (int it = 0; it < n; ++it) {
                    const int pv = L.PREV[(o << txl) + c];
                    if (pv < 0)
                        break;
                    const uint32_t wp = L.G[(pv << txl) + c];
                    if (fval(wp >> 2, pv, p0) > fval(wo >> 2, o, p0))
                        break;
                    o = pv;
                    wo = wp;
                }
                int nx_ = L.NEXT[(o << txl) + c];
                uint32_t wn = nx_ >= 0 ? L.G[(nx_ << txl) + c] : 0u;
                for (int p = p0; p < p1; ++p) {
                    for (int it = 0; it < n && nx_ >= 0 && fval(wn >> 2, nx_, p) < fval(wo >> 2, o, p); ++it) {
                        o = nx_;
                        wo = wn;
                        nx_ = L.NEXT[(o << txl) + c];
                        wn = nx_ >= 0 ? L.G[(nx_ << txl) + c] : 0u;
                    }
                    const int d = p - o;
                    const uint32_t word = wo + ((uint32_t)(d * d) << 2);
                    const int64_t gi = base + (int64_t)p * stride + c;
                    if (a.write_words)
                        a.w[gi] = word;
                    if (EPI)
                        interp_store(gi, word, a.w1, a.xq, a.out, a.eta_eb, a.power, a.td2, a.tw);
                }
            }
        }
    }
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

template <int AXIS, bool EPI, int M>
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
            L.G[L.at(cc, r)] = (x0 + cc < a.nx) ? a.w[base + (int64_t)r * stride + cc] : QAI_WORD_INF;
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

        // coalesced store (and step E when this is the last pass)
        for (int i = tid; i < total; i += blockDim.x) {
            const int r = i >> txl, cc = i & (Tx - 1);
            if (x0 + cc >= a.nx)
                continue;
            const uint32_t word = L.G[L.at(cc, r)];
            const int64_t gi = base + (int64_t)r * stride + cc;
            if (a.write_words)
                a.w[gi] = word;
            if (EPI)
                interp_store(gi, word, a.w1, a.xq, a.out, a.eta_eb, a.power, a.td2, a.tw);
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
    for (int i = 0; i < 3; ++i) {
        t.env_tx_log2[i] = -1;
        t.env_algo[i] = 0;
    }
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
    // windowed variant: keep the staged tile within 32 KB
    int l = 4;
    while (l > 0 && (n << l) * 4 > 32 * 1024)
        --l;
    return l;
}

static size_t band_bytes(int n, int B, int Tx)
{
    return (size_t)n * Tx * 8 + (size_t)B * Tx * 8 + (size_t)Tx * 8 + 64;
}

// Band geometry of a line of n positions: at most 64 bands of m positions,
// Tx columns per tile so that the LDS image stays within about 80 KB (two
// workgroups per CU), never below one column.
void band_geometry(int n, int want_txl, int& m, int& B, int& txl, size_t& lds)
{
    m = (n + 63) / 64;
    if (m < 1)
        m = 1;
    B = (n + m - 1) / m;
    txl = want_txl >= 0 ? want_txl : 4;
    while (txl > 0 && band_bytes(n, B, 1 << txl) > 80 * 1024)
        --txl;
    lds = band_bytes(n, B, 1 << txl);
}

template <int AXIS, bool EPI>
static hipError_t launch_band_t(EnvArgs a, int m, int B, size_t lds, int threads, uint32_t grid, hipStream_t s)
{
    static bool attr_done = false;
    if (lds > 64 * 1024 && !attr_done) {
        hipError_t e = hipFuncSetAttribute((const void*)k_env_band<AXIS, EPI>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds < 160 * 1024 ? 160 * 1024 : (int)lds);
        if (e != hipSuccess)
            return e;
        attr_done = true;
    }
    hipLaunchKernelGGL((k_env_band<AXIS, EPI>), dim3(grid), dim3(threads), lds, s, a, m, B);
    return hipGetLastError();
}


template <int AXIS, bool EPI, int M>
static hipError_t launch_band2_t(EnvArgs a, int lb, size_t lds, int threads, uint32_t grid, hipStream_t s)
{
    static bool attr_done = false;
    if (lds > 64 * 1024 && !attr_done) {
        hipError_t e = hipFuncSetAttribute((const void*)k_env_band2<AXIS, EPI, M>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess)
            return e;
        attr_done = true;
    }
    hipLaunchKernelGGL((k_env_band2<AXIS, EPI, M>), dim3(grid), dim3(threads), lds, s, a, lb);
    return hipGetLastError();
}

template <int AXIS, bool EPI>
static hipError_t launch_band2_m(EnvArgs a, int M, int lb, size_t lds, int threads, uint32_t grid, hipStream_t s)
{
    switch (M) {
    case 8: return launch_band2_t<AXIS, EPI, 8>(a, lb, lds, threads, grid, s);
    case 16: return launch_band2_t<AXIS, EPI, 16>(a, lb, lds, threads, grid, s);
    case 32: return launch_band2_t<AXIS, EPI, 32>(a, lb, lds, threads, grid, s);
    default: return launch_band2_t<AXIS, EPI, 64>(a, lb, lds, threads, grid, s);
    }
}

// Geometry of the wave-per-column variant: bands of M = max(8, 2^k) positions
// with at most 64 bands, B = 2^lb bands per column, Tx columns per tile
// (the LDS image is 8 bytes per padded position).
void band2_geometry(int n, int want_txl, int& M, int& lb, int& txl, size_t& lds)
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
    // a tile must fill whole wavefronts: Tx * B >= 64
    while ((B << txl) < 64)
        ++txl;
    lds = (size_t)(B * (M + 1) + 1) * (1 << txl) * 8;
}

hipError_t launch_band2(int axis, bool epi, EnvArgs a, const Tuning& t, hipStream_t s)
{
    const int n = (int)(axis == 1 ? a.ny : a.nz);
    int M, lb, txl;
    size_t lds;
    band2_geometry(n, t.env_tx_log2[axis], M, lb, txl, lds);
    a.tx_log2 = txl;
    const int64_t nxb = (a.nx + (1 << txl) - 1) >> txl;
    a.ntiles = (uint64_t)(nxb * (axis == 1 ? a.nz : a.ny));
    const uint32_t grid = grid_cap(a.ntiles, 1u << 20);
    const int threads = (1 << lb) << txl;
    if (axis == 1)
        return epi ? launch_band2_m<1, true>(a, M, lb, lds, threads, grid, s)
                   : launch_band2_m<1, false>(a, M, lb, lds, threads, grid, s);
    return epi ? launch_band2_m<2, true>(a, M, lb, lds, threads, grid, s)
               : launch_band2_m<2, false>(a, M, lb, lds, threads, grid, s);
}

hipError_t launch_env(int axis, bool epi, EnvArgs a, const Tuning& t, hipStream_t s)
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
        if (axis == 1) {
            if (epi) hipLaunchKernelGGL((k_env_window<1, true>), dim3(grid), blk, shm, s, a);
            else hipLaunchKernelGGL((k_env_window<1, false>), dim3(grid), blk, shm, s, a);
        } else {
            if (epi) hipLaunchKernelGGL((k_env_window<2, true>), dim3(grid), blk, shm, s, a);
            else hipLaunchKernelGGL((k_env_window<2, false>), dim3(grid), blk, shm, s, a);
        }
        return hipGetLastError();
    }
    if (n <= 64 * 32 && t.env_algo[axis] != 2)
        return launch_band2(axis, epi, a, t, s);
    int m, B, txl;
    size_t lds;
    band_geometry((int)n, t.env_tx_log2[axis], m, B, txl, lds);
    a.tx_log2 = txl;
    const int64_t nxb = (a.nx + (1 << txl) - 1) >> txl;
    a.ntiles = (uint64_t)(nxb * (axis == 1 ? a.nz : a.ny));
    const uint32_t grid = grid_cap(a.ntiles, 1u << 20);
    int threads = ((B << txl) + 63) / 64 * 64;
    if (axis == 1)
        return epi ? launch_band_t<1, true>(a, m, B, lds, threads, grid, s)
                   : launch_band_t<1, false>(a, m, B, lds, threads, grid, s);
    return epi ? launch_band_t<2, true>(a, m, B, lds, threads, grid, s)
               : launch_band_t<2, false>(a, m, B, lds, threads, grid, s);
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
