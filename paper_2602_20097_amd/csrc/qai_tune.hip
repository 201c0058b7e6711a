// qai_tune.hip -- launch-setting autotuner and its per-shape cache.
//
// Every setting (pass algorithm per axis, line-tile shape and workgroup size of
// the windowed passes, seed variant and z-march) computes the same exact
// transforms, so tuning changes only time.  The tuner times the candidates on
// one field in two rounds: first the pass algorithms with the seed variants,
// then, for the winner, the line-tile shapes of every pass it runs as the
// windowed search.  Results are kept per shape; the plain entry points use a
// shape's entry while the process-wide setting is the built-in default, and
// the cache can be written to and read from a text file.
#include <stdio.h>
#include <string.h>

#include <array>
#include <map>
#include <mutex>
#include <vector>

#include "qai.h"
#include "qai_device.h"
#include "qai_kernels.h"

using namespace qai::api;

namespace qai {
namespace {

std::mutex g_cache_mu;
std::map<std::array<int64_t, 3>, Tuning> g_cache;

std::array<int64_t, 3> key_of(const int64_t d[3]) { return {d[0], d[1], d[2]}; }

// The y-pass variants with the per-voxel direct search (algorithm 5) for a
// field whose y pass has fewer than 256 tiles of 64 columns; none otherwise.
std::vector<Tuning> few_tile_variants(const Tuning& base, int64_t nz, int64_t ny, int64_t nx)
{
    std::vector<Tuning> out;
    if (ny <= 1 || ((nx + 63) / 64) * nz >= 256)
        return out;
    const int e1s[2] = {-1, 5}, e2s[2] = {-1, 5};
    for (int a : e1s)
        for (int b : e2s) {
            if (a != 5 && b != 5)
                continue;
            Tuning t = base;
            t.edt1_algo[1] = a;
            t.env_algo[1] = b;
            out.push_back(t);
        }
    return out;
}

// Round 1: pass algorithms of both EDTs (automatic, the streaming kernel of
// each EDT, the windowed search, the banded envelope for the second EDT's y
// pass) times the seed variants.
std::vector<Tuning> round1(const Tuning& base, int64_t nz, int64_t ny, int64_t nx)
{
    std::vector<Tuning> out;
    // second EDT (y, z): automatic, per-lane envelope, windowed search, and the
    // banded envelope for the y pass ahead of the needed-voxel search
    const int e1s[3] = {-1, 4, 1}, e2s[4][2] = {{-1, -1}, {3, 3}, {1, 1}, {2, -1}};
    const int seeds[3][2] = {{0, 16}, {0, 32}, {4, 16}};
    for (int a : e1s)
        for (auto& b : e2s)
            for (auto& sd : seeds) {
                if (sd[0] == 0 && nx > kSeedLaneMaxX)
                    continue; // the register seed variant's longest line
                Tuning t = base;
                for (int k = 1; k < 3; ++k) {
                    t.edt1_algo[k] = a;
                    t.env_algo[k] = b[k - 1];
                }
                t.seed_ty = sd[0];
                t.seed_tz = sd[1];
                out.push_back(t);
            }
    // a y pass with few column tiles (a 2-D field): also the per-voxel direct
    // search for either EDT's y pass, the one choice that fills the GPU there
    for (const Tuning& t0 : few_tile_variants(base, nz, ny, nx)) {
        for (auto& sd : seeds) {
            if (sd[0] == 0 && nx > kSeedLaneMaxX)
                continue;
            Tuning t = t0;
            t.seed_ty = sd[0];
            t.seed_tz = sd[1];
            out.push_back(t);
        }
    }
    return out;
}

// Round 2: line-tile shapes (x-columns per tile, 2^tile_log2) and workgroup
// sizes of the windowed search, on the axes where the winner runs it.
std::vector<Tuning> round2(const Tuning& win, int64_t nz, int64_t ny, int64_t nx)
{
    std::vector<Tuning> out;
    bool uses[3] = {false, false, false};
    for (int a = 1; a <= 2; ++a) {
        const int64_t ext = a == 1 ? ny : nz;
        if (ext <= 1)
            continue;
        uses[a] = resolve_algo(win.edt1_algo[a], true, a, nz, ny, nx) == 1 ||
                  resolve_algo(win.env_algo[a], false, a, nz, ny, nx) == 1;
    }
    if (!uses[1] && !uses[2])
        return out;
    const int tiles[5] = {-1, 3, 4, 5, 6};
    const int threads[4] = {128, 256, 512, 1024};
    for (int tl : tiles)
        for (int th : threads) {
            Tuning t = win;
            for (int a = 1; a <= 2; ++a)
                if (uses[a])
                    t.env_tx_log2[a] = tl;
            t.env_threads = th;
            out.push_back(t);
        }
    return out;
}

hipError_t time_run(Plan1& pl, const Tuning& t, hipStream_t s, hipEvent_t a, hipEvent_t b, float& ms)
{
    hipError_t e = run_plain(pl, t, s); // warm-up
    if (e != hipSuccess)
        return e;
    if ((e = hipEventRecord(a, s)) != hipSuccess)
        return e;
    for (int r = 0; r < 2; ++r)
        if ((e = run_plain(pl, t, s)) != hipSuccess)
            return e;
    if ((e = hipEventRecord(b, s)) != hipSuccess)
        return e;
    if ((e = hipEventSynchronize(b)) != hipSuccess)
        return e;
    return hipEventElapsedTime(&ms, a, b);
}

} // namespace

bool cache_lookup(const int64_t dims[3], Tuning& t)
{
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_cache.find(key_of(dims));
    if (it == g_cache.end())
        return false;
    t = it->second;
    return true;
}

void cache_store(const int64_t dims[3], const Tuning& t)
{
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_cache[key_of(dims)] = t;
}

hipError_t tune_field(Plan1& p, const Tuning& base, hipStream_t s, Tuning& best, int* n_timed)
{
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess)
        e = hipEventCreate(&b);
    if (e != hipSuccess) {
        if (a)
            (void)hipEventDestroy(a);
        return e;
    }
    float best_ms = 1e30f;
    best = base;
    int timed = 0;
    for (int round = 0; round < 2 && e == hipSuccess; ++round) {
        const std::vector<Tuning> cands =
            round == 0 ? round1(base, p.nz, p.ny, p.nx) : round2(best, p.nz, p.ny, p.nx);
        for (const Tuning& t : cands) {
            float ms = 0.0f;
            if ((e = time_run(p, t, s, a, b, ms)) != hipSuccess)
                break;
            ++timed;
            if (ms < best_ms) {
                best_ms = ms;
                best = t;
            }
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (n_timed)
        *n_timed = timed;
    return e;
}

// Variants of a shape's setting for one field: the pass algorithms of both
// EDTs, whose best choice follows the field's boundary density (sparse
// boundaries: longer distances) more than its shape.
hipError_t refine_field(Plan1& p, const Tuning& shape_best, hipStream_t s, Tuning& best)
{
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess)
        e = hipEventCreate(&b);
    if (e != hipSuccess) {
        if (a)
            (void)hipEventDestroy(a);
        return e;
    }
    std::vector<Tuning> cands;
    cands.push_back(shape_best);
    const int e1s[2] = {-1, 1}, e2s[4][2] = {{-1, -1}, {3, 3}, {1, 1}, {2, -1}};
    for (int x : e1s)
        for (auto& y : e2s) {
            Tuning t = shape_best;
            for (int k = 1; k < 3; ++k) {
                t.edt1_algo[k] = x;
                t.env_algo[k] = y[k - 1];
            }
            cands.push_back(t);
        }
    for (const Tuning& t : few_tile_variants(shape_best, p.nz, p.ny, p.nx))
        cands.push_back(t);
    float best_ms = 1e30f;
    best = shape_best;
    for (const Tuning& t : cands) {
        float ms = 0.0f;
        if ((e = time_run(p, t, s, a, b, ms)) != hipSuccess)
            break;
        if (ms < best_ms) {
            best_ms = ms;
            best = t;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return e;
}

} // namespace qai

namespace {

// One line per shape: nz ny nx, then the setting's fields in the order of
// qai_tuning (force_wide excluded: the cache holds 32-bit index settings).
constexpr const char* kCacheHeader = "qai-tuning-cache 1";

} // namespace

extern "C" {

int qai_autotune(const float* field, const int64_t dims[3], float eb, void* ws, size_t ws_bytes, float* out,
                 void* stream, qai_tuning* best)
{
    clear_error();
    int64_t n;
    int rc = check_dims(dims, &n);
    if (rc)
        return rc;
    if (!field || !out)
        return fail(QAI_EINVAL, "field and out must be device pointers");
    if ((rc = check_eb(eb)))
        return rc;
    const size_t need = qai_workspace_bytes(dims);
    if (!ws || ws_bytes < need)
        return fail(QAI_ENOWS, "workspace of %zu bytes needed, %zu given", need, ws ? ws_bytes : (size_t)0);
    if (((uintptr_t)ws & 255u) != 0)
        return fail(QAI_ENOWS, "workspace must be 256-byte aligned");
    if (out < field + n && field < out + n)
        return fail(QAI_EINVAL, "autotuning needs an output apart from the field");
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
    pl.eta = 0.9f;
    pl.power = 1.0f;
    ws_buffers(ws, pl);
    if ((e = qai::aux_for(dev, pl.aux)) != hipSuccess)
        return fail_hip(e, "side stream");
    std::lock_guard<std::mutex> lk(pl.aux->mu);
    qai::Tuning base;
    qai::default_tuning(base);
    qai::Tuning pick;
    prof_suppress(true);
    e = qai::tune_field(pl, base, (hipStream_t)stream, pick, nullptr);
    prof_suppress(false);
    if (e != hipSuccess)
        return fail_hip(e, "autotune run");
    qai::cache_store(dims, pick);
    if (best)
        tuning_to_abi(pick, best);
    return QAI_OK;
}

int qai_tuning_cache_clear(void)
{
    clear_error();
    std::lock_guard<std::mutex> lk(qai::g_cache_mu);
    qai::g_cache.clear();
    return QAI_OK;
}

int qai_tuning_cache_size(void)
{
    std::lock_guard<std::mutex> lk(qai::g_cache_mu);
    return (int)qai::g_cache.size();
}

int qai_tuning_cache_save(const char* path)
{
    clear_error();
    if (!path)
        return fail(QAI_EINVAL, "path is NULL");
    std::map<std::array<int64_t, 3>, qai::Tuning> snap;
    {
        std::lock_guard<std::mutex> lk(qai::g_cache_mu);
        snap = qai::g_cache;
    }
    FILE* f = fopen(path, "w");
    if (!f)
        return fail(QAI_EINVAL, "cannot write %s", path);
    fprintf(f, "%s\n", kCacheHeader);
    for (const auto& kv : snap) {
        qai_tuning t;
        tuning_to_abi(kv.second, &t);
        fprintf(f, "%lld %lld %lld %d %d %d %d %d %d %d %d %d %d %d\n", (long long)kv.first[0],
                (long long)kv.first[1], (long long)kv.first[2], t.edt1_algo[0], t.edt1_algo[1], t.edt2_algo[0],
                t.edt2_algo[1], t.edt1_ring, t.edt2_ring, t.tile_log2[0], t.tile_log2[1], t.seed_rows,
                t.seed_planes, t.window_threads);
    }
    const bool ok = ferror(f) == 0;
    if (fclose(f) != 0 || !ok)
        return fail(QAI_EINVAL, "error writing %s", path);
    return QAI_OK;
}

int qai_tuning_cache_load(const char* path)
{
    clear_error();
    if (!path)
        return fail(QAI_EINVAL, "path is NULL");
    FILE* f = fopen(path, "r");
    if (!f)
        return fail(QAI_EINVAL, "cannot read %s", path);
    char line[512];
    if (!fgets(line, sizeof line, f) || strncmp(line, kCacheHeader, strlen(kCacheHeader)) != 0) {
        fclose(f);
        return fail(QAI_EINVAL, "%s is not a tuning cache", path);
    }
    std::vector<std::pair<std::array<int64_t, 3>, qai::Tuning>> rows;
    int lineno = 1;
    while (fgets(line, sizeof line, f)) {
        ++lineno;
        long long d[3];
        qai_tuning t = {};
        const int k = sscanf(line, "%lld %lld %lld %d %d %d %d %d %d %d %d %d %d %d", &d[0], &d[1], &d[2],
                             &t.edt1_algo[0], &t.edt1_algo[1], &t.edt2_algo[0], &t.edt2_algo[1], &t.edt1_ring,
                             &t.edt2_ring, &t.tile_log2[0], &t.tile_log2[1], &t.seed_rows, &t.seed_planes,
                             &t.window_threads);
        if (k == EOF || (k == 0 && line[0] == '\n'))
            continue;
        if (k != 14) {
            fclose(f);
            return fail(QAI_EINVAL, "%s line %d: 14 fields expected", path, lineno);
        }
        const int64_t dims[3] = {d[0], d[1], d[2]};
        int64_t n;
        if (check_dims(dims, &n)) {
            fclose(f);
            return fail(QAI_EINVAL, "%s line %d: bad extents", path, lineno);
        }
        qai::Tuning q;
        if (abi_to_tuning(&t, q)) {
            fclose(f);
            return fail(QAI_EINVAL, "%s line %d: %s", path, lineno, qai_last_error());
        }
        rows.push_back({{d[0], d[1], d[2]}, q});
    }
    fclose(f);
    std::lock_guard<std::mutex> lk(qai::g_cache_mu);
    for (const auto& r : rows)
        qai::g_cache[r.first] = r.second;
    return QAI_OK;
}

} // extern "C"
