/*
 * qai_oracle.c -- plain, slow, FP64 CPU reference of the quantization-aware
 * interpolation (QAI) post-pass of Jiao et al., "Mitigating Artifacts in
 * Pre-quantization Based Scientific Data Compressors with Quantization-aware
 * Interpolation" (arXiv 2602.20097).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker the GPU library is
 * compared against.  Only the test-suite, the package's smoke check and the
 * CPU-baseline leg of the benchmark may load it; the library never does.  It
 * shares no source, header, table or helper with the GPU path.
 *
 * It follows the paper's algorithms in their order and notation:
 *   Step A  Algorithm 2  GetBoundaryAndSignMap3D        -> B1, S_B
 *   Step B  Algorithm 1  VoronoiEDT, once per axis       -> Dist1, I1
 *   Step C  Algorithm 3  PropagateSignsAndConstructSignMap -> S, B2
 *   Step D  Algorithm 1  VoronoiEDT on B2 (no indices)   -> Dist2
 *   Step E  Section V-E  inverse-distance weighting      -> C, D'' = D' + C
 *   chained as in Algorithm 4 (Distance-Based Compensation).
 * Floating point is double throughout (the single-precision input and the
 * single-precision parameters eb, eta, power are widened exactly); the EDT
 * runs in int64.  Loops are parallelised with OpenMP over independent voxels
 * or lines only; no step is blocked, fused or reordered.
 *
 * Readings of points the paper leaves open (each is also listed with the
 * design notes of the repository):
 *   - q is recovered from the decompressed value as rintf(x'/(2 eb)) in
 *     single precision, the precision of the data (Section VII-B); both sides
 *     of a parity check take that integer decision the same way.
 *   - Axes of extent 1 carry no neighbours and no edge exclusion; an axis of
 *     extent n > 1 is interior for coordinates 1..n-2 (Algorithm 2's loops).
 *   - "q differs from any of its 6 neighbours" means: from at least one.
 *   - The boundary sign is sgn(q_nb - q) for the first differing neighbour in
 *     the order +x, -x, +y, -y, +z, -z (x is the fastest axis); this makes
 *     the lower side of a q -> q+1 transition positive and the upper side
 *     negative, as Section V (error sign flipping) describes.
 *   - The gradient test uses absolute central differences, |q+ - q-|/2 >= 1.
 *   - The EDT passes run along x, then y, then z.  With Algorithm 1's strict
 *     inequalities each pass keeps the lowest coordinate among tied sites, so
 *     I1 is the smallest linear index among the nearest boundary voxels.
 *   - B2 holds interior voxels that are not in B1 and whose propagated sign
 *     differs from a 6-neighbour's (GetBoundary done the Algorithm 2 way).
 *   - Interpolation: k1 = sqrt(Dist1^2), k2 = sqrt(Dist2^2) (Euclidean);
 *     w = 1 on B1, w = 0 on B2, w = 1 when B2 is empty; otherwise
 *     w = k1^-p / (k1^-p + k2^-p), which for p = 1 is the paper's
 *     (1/k1)/(1/k1 + 1/k2).  C = w * S * eta * eb.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_INF INT64_MAX

/* status bits returned by orc_qai */
#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_EQRANGE (-3)

typedef struct {
    int64_t n[3];      /* extents: n[0] = x (fastest), n[1] = y, n[2] = z */
    int64_t stride[3]; /* element strides along x, y, z */
    int64_t total;
} grid_t;

static grid_t make_grid(int64_t nz, int64_t ny, int64_t nx)
{
    grid_t g;
    g.n[0] = nx;
    g.n[1] = ny;
    g.n[2] = nz;
    g.stride[0] = 1;
    g.stride[1] = nx;
    g.stride[2] = nx * ny;
    g.total = nx * ny * nz;
    return g;
}

static void coords(const grid_t* g, int64_t i, int64_t c[3])
{
    c[0] = i % g->n[0];
    c[1] = (i / g->n[0]) % g->n[1];
    c[2] = i / (g->n[0] * g->n[1]);
}

/* A voxel is interior when every axis of extent > 1 has 1 <= c <= n-2
 * (Algorithm 2 visits i = 1..d0-2, j = 1..d1-2, k = 1..d2-2). */
static int is_interior(const grid_t* g, const int64_t c[3])
{
    for (int a = 0; a < 3; ++a)
        if (g->n[a] > 1 && (c[a] < 1 || c[a] > g->n[a] - 2))
            return 0;
    return 1;
}

/* Eq. 1 inverted: d' = 2 q eps  =>  q = round(d' / 2 eps), in single precision. */
int orc_recover_q(const float* xq, int64_t n, float eb, int32_t* q)
{
    int bad = 0;
#pragma omp parallel for reduction(| : bad)
    for (int64_t i = 0; i < n; ++i) {
        float t = xq[i] / (2.0f * eb);
        if (!(fabsf(t) <= 2097152.0f)) { /* |q| <= 2^21 */
            bad = 1;
            q[i] = 0;
            continue;
        }
        q[i] = (int32_t)rintf(t);
    }
    return bad ? ORC_EQRANGE : ORC_OK;
}

/* Algorithm 2, GetBoundaryAndSignMap3D: B[i] = 1 at quantization boundaries,
 * S[i] = sign of the quantization error estimated there. */
void orc_boundary_sign(const int32_t* q, int64_t nz, int64_t ny, int64_t nx, uint8_t* B, int8_t* S)
{
    grid_t g = make_grid(nz, ny, nx);
#pragma omp parallel for
    for (int64_t i = 0; i < g.total; ++i) {
        int64_t c[3];
        B[i] = 0;
        S[i] = 0;
        coords(&g, i, c);
        if (!is_interior(&g, c))
            continue;
        int64_t qc = q[i];
        int64_t first_diff = 0;
        int found = 0;
        for (int a = 0; a < 3 && !found; ++a) {
            if (g.n[a] == 1)
                continue;
            int64_t plus = q[i + g.stride[a]];
            int64_t minus = q[i - g.stride[a]];
            if (plus != qc) {
                first_diff = plus - qc;
                found = 1;
            } else if (minus != qc) {
                first_diff = minus - qc;
                found = 1;
            }
        }
        if (!found)
            continue;
        B[i] = 1;                                   /* in B1 */
        S[i] = (int8_t)(first_diff > 0 ? 1 : -1);   /* sign of (first differing neighbour - q) */
        for (int a = 0; a < 3; ++a) {               /* half the index jump across the voxel, per axis */
            if (g.n[a] == 1)
                continue;
            double grad = fabs((double)((int64_t)q[i + g.stride[a]] - (int64_t)q[i - g.stride[a]])) / 2.0;
            if (grad >= 1.0)
                S[i] = 0;                           /* steep: the error sign is not predictable */
        }
    }
}

/* The squared distance transform along one line is Eq. 2 restricted to the
 * line: D(i) = min over sites j of f(j) + (i - j)^2, where the sites are the
 * entries with f(j) finite.  Seen as functions of i, the terms are parabolas
 * P_j of one common curvature, so each parabola is the minimum on at most one
 * interval, and those intervals come in the order of the sites.  Algorithm 1
 * (Section III-B) keeps the parabolas that are the minimum somewhere, in site
 * order, and then reads the minimum off that list row by row.
 *
 * Crossing points: P_v (v > u) drops below P_u for i beyond
 *   t(u, v) = (f(v) - f(u) + v^2 - u^2) / (2 (v - u)).
 * With u < v < w, P_v is the minimum nowhere between P_u and P_w when it only
 * drops below P_u after P_w has already dropped below it: t(u, v) > t(v, w).
 * Multiplied by 2 (v - u)(w - v) > 0 this is an integer comparison; it is the
 * same predicate as the paper's RemoveEDT (expand and collect the terms), and
 * like it, it keeps P_v when the two crossing points coincide. */
static int parabola_hidden(int64_t fu, int64_t u, int64_t fv, int64_t v, int64_t fw, int64_t w)
{
    const int64_t a = v - u, b = w - v;
    return b * (fv - fu + v * v - u * u) > a * (fw - fv + w * w - v * v);
}

/* Algorithm 1 on one line: D[base + i*stride], i = 0..n-1 (ORC_INF = not a
 * site).  Feature indices F (nullable) travel with their sites.  env_* are
 * scratch arrays of n entries holding the kept parabolas: value, position and
 * feature. */
static void voronoi_edt(int64_t* D, int64_t* F, int64_t base, int64_t stride, int64_t n,
                        int64_t* env_f, int64_t* env_pos, int64_t* env_feat)
{
    int64_t kept = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t fi = D[base + i * stride];
        if (fi == ORC_INF)
            continue;
        /* retire parabolas the new one hides behind their predecessors */
        while (kept >= 2 && parabola_hidden(env_f[kept - 2], env_pos[kept - 2], env_f[kept - 1], env_pos[kept - 1],
                                            fi, i))
            --kept;
        env_f[kept] = fi;
        env_pos[kept] = i;
        if (F)
            env_feat[kept] = F[base + i * stride];
        ++kept;
    }
    if (kept == 0)
        return; /* no site on the line: every entry stays ORC_INF */
    /* the minimum at row i comes from the current parabola; move on while the
     * next one is strictly lower there (a tie keeps the lower position) */
    int64_t cur = 0;
    for (int64_t i = 0; i < n; ++i) {
        while (cur + 1 < kept) {
            const int64_t here = env_f[cur] + (i - env_pos[cur]) * (i - env_pos[cur]);
            const int64_t next = env_f[cur + 1] + (i - env_pos[cur + 1]) * (i - env_pos[cur + 1]);
            if (!(next < here))
                break;
            ++cur;
        }
        D[base + i * stride] = env_f[cur] + (i - env_pos[cur]) * (i - env_pos[cur]);
        if (F)
            F[base + i * stride] = env_feat[cur];
    }
}

/* One VoronoiEDT pass along axis a over every line of the grid. */
static int edt_pass(int64_t* D, int64_t* F, const grid_t* g, int a)
{
    int64_t n = g->n[a];
    if (n == 1)
        return ORC_OK; /* a line of one voxel is left as it is */
    int64_t lines = g->total / n;
    int err = 0;
#pragma omp parallel reduction(| : err)
    {
        int64_t* sg = (int64_t*)malloc(sizeof(int64_t) * n);
        int64_t* sh = (int64_t*)malloc(sizeof(int64_t) * n);
        int64_t* sf = (int64_t*)malloc(sizeof(int64_t) * n);
        if (!sg || !sh || !sf) {
            err = 1;
        } else {
#pragma omp for
            for (int64_t L = 0; L < lines; ++L) {
                /* line L enumerates the two other axes, slower one outer */
                int64_t base;
                if (a == 0) {
                    base = L * g->n[0];
                } else if (a == 1) {
                    int64_t x = L % g->n[0], z = L / g->n[0];
                    base = z * g->stride[2] + x;
                } else {
                    base = L; /* (y, x) plane index */
                }
                voronoi_edt(D, F, base, g->stride[a], n, sg, sh, sf);
            }
        }
        free(sg);
        free(sh);
        free(sf);
    }
    return err ? ORC_ENOMEM : ORC_OK;
}

/* EuclideanDistanceTransform(B): squared distance of every voxel to the
 * nearest voxel with B = 1 (Eq. 2), and when F is given the linear index of
 * that voxel.  Passes along x, then y, then z.  No seed at all leaves every
 * distance at ORC_INF and every feature at -1. */
int orc_edt(const uint8_t* B, int64_t nz, int64_t ny, int64_t nx, int64_t* D, int64_t* F)
{
    grid_t g = make_grid(nz, ny, nx);
#pragma omp parallel for
    for (int64_t i = 0; i < g.total; ++i) {
        D[i] = B[i] ? 0 : ORC_INF;
        if (F)
            F[i] = B[i] ? i : -1;
    }
    for (int a = 0; a < 3; ++a) {
        int rc = edt_pass(D, F, &g, a);
        if (rc)
            return rc;
    }
    return ORC_OK;
}

/* Algorithm 3, PropagateSignsAndConstructSignMap: S takes the boundary sign of
 * the nearest boundary voxel I_B; B2 = GetBoundary(S) restricted to interior
 * voxels outside B1. */
void orc_propagate(const uint8_t* B1, const int8_t* SB, const int64_t* IB, int64_t nz, int64_t ny,
                   int64_t nx, int8_t* S, uint8_t* B2)
{
    grid_t g = make_grid(nz, ny, nx);
#pragma omp parallel for
    for (int64_t i = 0; i < g.total; ++i) {
        if (B1[i] == 1)
            S[i] = SB[i];
        else
            S[i] = IB[i] >= 0 ? SB[IB[i]] : 0; /* no boundary anywhere: no sign */
    }
#pragma omp parallel for
    for (int64_t i = 0; i < g.total; ++i) {
        int64_t c[3];
        B2[i] = 0;
        coords(&g, i, c);
        if (B1[i] || !is_interior(&g, c))
            continue;
        for (int a = 0; a < 3; ++a) {
            if (g.n[a] == 1)
                continue;
            if (S[i + g.stride[a]] != S[i] || S[i - g.stride[a]] != S[i]) {
                B2[i] = 1;
                break;
            }
        }
    }
}

/* Interpolate(dist1, dist2, S, eta eps) of Algorithm 4 with the IDW weight of
 * Section V-E, generalised to power p (p = 1 is the paper's weight).
 * d1sq/d2sq == ORC_INF means no boundary of that kind exists. */
static double idw_weight(int64_t d1sq, int64_t d2sq, double p)
{
    double k1 = d1sq == ORC_INF ? INFINITY : sqrt((double)d1sq);
    double k2 = d2sq == ORC_INF ? INFINITY : sqrt((double)d2sq);
    if (k1 == 0.0)
        return 1.0; /* on a quantization boundary */
    if (k2 == 0.0)
        return 0.0; /* on a sign-flipping boundary */
    if (isinf(k2))
        return 1.0; /* no sign-flipping boundary: 1/k2 = 0 */
    if (isinf(k1))
        return 0.0;
    if (p == 1.0)
        return (1.0 / k1) / (1.0 / k1 + 1.0 / k2);
    return pow(k1, -p) / (pow(k1, -p) + pow(k2, -p));
}

void orc_interp(const float* xq, const int64_t* D1, const int64_t* D2, const int8_t* S, int64_t n,
                float eb, float eta, float power, double* out, double* w_out)
{
    double e = (double)eta * (double)eb;
#pragma omp parallel for
    for (int64_t i = 0; i < n; ++i) {
        double w = idw_weight(D1[i], D2[i], (double)power);
        double C = w * (double)S[i] * e;
        out[i] = (double)xq[i] + C;  /* D'' = D' + C */
        if (w_out)
            w_out[i] = w;
    }
}

/* Algorithm 4, Distance-Based Compensation, with every intermediate exposed.
 * Required: xq, out.  Every other output pointer may be NULL. */
int orc_qai(const float* xq, int64_t nz, int64_t ny, int64_t nx, float eb, float eta, float power,
            double* out, int32_t* q_o, uint8_t* b1_o, int8_t* sb_o, int64_t* d1_o, int64_t* i1_o,
            int8_t* s_o, uint8_t* b2_o, int64_t* d2_o, double* w_o)
{
    if (!xq || !out || nz < 1 || ny < 1 || nx < 1 || !(eb > 0.0f) || !isfinite(eb))
        return ORC_EINVAL;
    int64_t n = nz * ny * nx;
    int32_t* q = q_o ? q_o : (int32_t*)malloc(sizeof(int32_t) * n);
    uint8_t* B1 = b1_o ? b1_o : (uint8_t*)malloc(n);
    int8_t* SB = sb_o ? sb_o : (int8_t*)malloc(n);
    int64_t* D1 = d1_o ? d1_o : (int64_t*)malloc(sizeof(int64_t) * n);
    int64_t* I1 = i1_o ? i1_o : (int64_t*)malloc(sizeof(int64_t) * n);
    int8_t* S = s_o ? s_o : (int8_t*)malloc(n);
    uint8_t* B2 = b2_o ? b2_o : (uint8_t*)malloc(n);
    int64_t* D2 = d2_o ? d2_o : (int64_t*)malloc(sizeof(int64_t) * n);
    int rc = ORC_OK;
    if (!q || !B1 || !SB || !D1 || !I1 || !S || !B2 || !D2) {
        rc = ORC_ENOMEM;
        goto done;
    }
    rc = orc_recover_q(xq, n, eb, q);
    if (rc)
        goto done;
    orc_boundary_sign(q, nz, ny, nx, B1, SB);               /* step A */
    rc = orc_edt(B1, nz, ny, nx, D1, I1);                   /* step B */
    if (rc)
        goto done;
    orc_propagate(B1, SB, I1, nz, ny, nx, S, B2);           /* step C */
    rc = orc_edt(B2, nz, ny, nx, D2, NULL);                 /* step D */
    if (rc)
        goto done;
    orc_interp(xq, D1, D2, S, n, eb, eta, power, out, w_o); /* step E */
done:
    if (!q_o) free(q);
    if (!b1_o) free(B1);
    if (!sb_o) free(SB);
    if (!d1_o) free(D1);
    if (!i1_o) free(I1);
    if (!s_o) free(S);
    if (!b2_o) free(B2);
    if (!d2_o) free(D2);
    return rc;
}

int orc_max_threads(void);
#ifdef _OPENMP
#include <omp.h>
int orc_max_threads(void) { return omp_get_max_threads(); }
#else
int orc_max_threads(void) { return 1; }
#endif
