// qai_kernels.h -- kernel argument blocks and the host-side launchers of the
// plain post-pass (used by the C ABI, the batched plan and the autotuner).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <mutex>

#include "qai.h"

namespace qai {

// Largest workgroup the kernel fn was compiled for (its __launch_bounds__, as
// the runtime reports it), cached per kernel; 0 if the runtime cannot tell.
int kernel_block_limit(const void* fn);

template <typename T>
struct same_type {
    using type = T;
};

// Every kernel of the library is launched through here: a workgroup larger
// than the kernel's compiled bound (which the hardware would run with too few
// registers per lane) is refused on the host with hipErrorInvalidConfiguration
// before anything is enqueued.
template <typename... P>
hipError_t launch_checked(void (*fn)(P...), dim3 grid, dim3 block, size_t shm, hipStream_t s,
                          typename same_type<P>::type... args)
{
    const int64_t threads = (int64_t)block.x * block.y * block.z;
    const int lim = kernel_block_limit((const void*)fn);
    if (lim <= 0 || threads > lim || threads < 1 || grid.x == 0)
        return hipErrorInvalidConfiguration;
    void* argv[] = {(void*)&args...};
    const hipError_t e = hipLaunchKernel((const void*)fn, grid, block, argv, shm, s);
    return e != hipSuccess ? e : hipGetLastError();
}

// Stage A (+ the first EDT pass) or stage C (+ the first pass of the second
// EDT): a 6-neighbour stencil marks the sites, then a scan along x gives each
// voxel its nearest site on its x-line.
struct SeedArgs {
    const float* xq;      // mode 0 input: decompressed field
    const uint32_t* w1;   // mode 1 input: final words of the first EDT
    uint32_t* wout;       // output words
    int64_t nx, ny, nz;
    float inv2eb, two_eb; // 1/(2 eb) rounded, 2 eb exact
    uint32_t* status;
    int32_t* tq;          // taps (nullable)
    uint8_t* tb1;
    int8_t* tsb;
    int8_t* ts;
    int32_t* td1;
    uint8_t* tb2;
    uint64_t ngroups;     // line groups (one line per wave)
    int waves;            // waves per workgroup
    unsigned long long* b1count; // mode 0, k_seed_lane only (nullable): an estimate of the B1 voxels
                                 // (a 1-in-V sample, scaled) is added here
    // coded indices (k_seed_lane mode 2): segments of 32 voxels per x-row
    const int32_t* cbase;         // first index of each segment
    const uint64_t* cmeta;        // (first payload word << 8) | width of its differences
    const uint32_t* cpay;         // the payload words
    uint32_t cpay_bytes;          // their size: reads past it return 0 (buffer loads)
    int64_t segs_row;             // segments per x-row, ceil(nx / 32)
    float* xout;                  // receives x' = 2 eb q of every voxel
};

// One lower-envelope pass along y (axis 1) or z (axis 2) over packed words,
// optionally finished by the interpolation of step E.
struct EnvArgs {
    const uint32_t* win;  // words before the pass
    uint32_t* w;          // words after the pass (may equal win for the tiled variants)
    int64_t nx, ny, nz;
    int tx_log2;          // columns per tile = 1 << tx_log2
    uint64_t ntiles;
    const uint32_t* gate; // when set, the pass runs only if *gate != 0 (windowed and streaming outward searches)
};

// Words of the workspace header for the fused y/z pass of the first EDT,
// cleared with the status word: QAI_WIDE_WORD is raised when some voxel's
// distance lies beyond the search disc (or the pass stands down), and the
// 64-bit estimate of the B1 voxels from the seed pass sits at QAI_B1_WORD.
// QAI_OVF_WORD is raised when the second EDT's y pass (per-lane envelope)
// finds a column whose live window outgrows its ring; the banded pass then
// recomputes the whole y pass (gated on the word).
#define QAI_WIDE_WORD 16
#define QAI_OVF_WORD 17
#define QAI_B1_WORD 18
#define QAI_OVFZ_WORD 20 // the same as QAI_OVF_WORD for a whole z pass of the second EDT
#define QAI_HEADER_WORDS 24

struct InterpArgs {
    const uint32_t* w1;
    const uint32_t* w2;
    const float* xq;
    float* out;
    int64_t n;
    float eta_eb, power;
    int32_t* td2;
    float* tw;
    const unsigned long long* only_sparse; // when set, runs only where sparse_b1 holds for this estimate
};

// Launch geometry chosen per pass (the autotuner overrides the defaults).
struct Tuning {
    int env_tx_log2[3];   // per axis (index 1 = y, 2 = z); -1 = default
    int env_algo[3];      // per axis: 0 = streaming envelope, 1 = windowed search, 2 = banded
    int stream_cap[3];    // per axis: live-stack ring entries of the streaming envelope, second EDT
    int edt1_cap[3];      // the same for the first EDT (16, 32 or 64)
    int edt1_algo[3];     // env_algo for the first EDT
    int env_threads;      // threads per workgroup of the windowed variant
    int seed_ty, seed_tz; // x-lines (waves) and z-planes per workgroup of the seed passes
    int force_wide;       // 1: take the 64-bit index/arithmetic variant wherever a kernel has one
};

void default_tuning(Tuning& t);

// The pass algorithm a choice of -1 (automatic) stands for on a field of this
// shape (axis 1 = y, 2 = z); an explicit choice is returned unchanged.
int resolve_algo(int want, bool first_edt, int axis, int64_t nz, int64_t ny, int64_t nx);

// Longest x-line of the register-resident seed pass (k_seed_lane): lines of
// up to 512 voxels take one wave, longer ones two, four or eight.
constexpr int64_t kSeedLaneMaxX = 4096;

struct Plan1;

// Per-shape tuning cache (filled by the autotuner, saved to and loaded from a
// text file).  cache_lookup returns false when the shape has no entry.
bool cache_lookup(const int64_t dims[3], Tuning& t);
void cache_store(const int64_t dims[3], const Tuning& t);
// Time the candidate settings on one field (its plan filled in) and return
// the fastest; base supplies the fields the candidates do not vary.
hipError_t tune_field(Plan1& p, const Tuning& base, hipStream_t s, Tuning& best, int* n_timed);
// Time the pass-algorithm variants of a shape's setting on one field (boundary
// density decides between them more than shape) and return the fastest.
hipError_t refine_field(Plan1& p, const Tuning& shape_best, hipStream_t s, Tuning& best);

// Host launchers: return hipSuccess or the launch error.
hipError_t launch_seed(int mode, const SeedArgs& a, hipStream_t s, int ty, int tz);
hipError_t launch_env(int axis, EnvArgs a, const Tuning& t, hipStream_t s);
hipError_t launch_interp(const InterpArgs& a, hipStream_t s);
hipError_t launch_clear(uint32_t* p, int n, hipStream_t s);

// The full plain post-pass on one field (stages in order).  ws_words points
// at 2*N words (w1 then w2), status at one word.
// Word buffers rotate through the passes: A, B and C hold N words each.  On
// return w1_final / w2_final point at the final words of the two EDTs.
// Coded quantization indices (qai_coded): segments of 32 voxels per x-row.
struct Coded {
    const int32_t* base;
    const uint64_t* meta;
    const uint32_t* payload;
    uint64_t payload_words;
};
bool coded_seed_supported(int64_t nx);
hipError_t launch_seed_coded(const SeedArgs& in, int tz, hipStream_t s);
// x' = 2 eb q of every voxel from the code (one wave per two segments)
hipError_t launch_decode(const Coded& c, int64_t nz, int64_t ny, int64_t nx, float two_eb, float* xq, hipStream_t s);

// A side stream and two events per device.  With one attached to a plan, the
// streaming part of step E (every voxel whose weight does not need the second
// EDT's z pass) runs on the side stream while the second EDT's y pass runs on
// the caller's stream, ordered by the events.  The caller holds mu from the
// plan's first launch to its last (the events are shared).
struct Aux {
    std::mutex mu;
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};
hipError_t aux_for(int dev, Aux*& out);
// True while s is being captured into a graph (or its state is unknown): the
// side stream is then left out, every launch stays on s.
bool stream_capturing(hipStream_t s);

struct Plan1 {
    const Coded* coded;   // when set, the indices come from this code and x' is written to out
    const float* xq;
    float* out;
    int64_t nz, ny, nx;
    float eb, eta, power;
    uint32_t* bufA;
    uint32_t* bufB;
    uint32_t* bufC;
    uint32_t* status;
    uint64_t* flags;      // fused final pass: one bit per voxel, see flag_bytes
    Aux* aux;             // when set (mu held), the overlap described at Aux
    qai_taps taps;
    const uint32_t* w1_final;
    const uint32_t* w2_final;
};
hipError_t run_plain(Plan1& p, const Tuning& t, hipStream_t s);
// The same in two halves: steps A and B, then (with the first EDT's words in
// buffer w1, which a caller may edit in between) steps C, D and E.
hipError_t run_part1(Plan1& p, const Tuning& t, hipStream_t s, int* w1);
hipError_t run_part2(Plan1& p, const Tuning& t, hipStream_t s, int w1);

// Bytes of the fused final pass's flag words for n voxels: one 64-bit word
// per 64 voxels, in blocks of 1024 voxels.
inline size_t flag_bytes(int64_t n) { return (size_t)((n + 1023) / 1024) * 128; }

// Words per distance-word buffer: the voxel count with ny rounded up to a
// multiple of 4, room for the blocked layout [z][y/4][x][y%4] in which the
// second EDT's y pass hands its result to the needed-voxel search.
inline int64_t word_capacity(int64_t nz, int64_t ny, int64_t nx) { return nz * ((ny + 3) / 4) * 4 * nx; }

// Stage-timing hooks (active when profiling is enabled).
void prof_begin(const char* name, hipStream_t s);
void prof_end(hipStream_t s);

// Host-side helpers of the C ABI shared by the plain and batched entry points.
namespace api {
constexpr size_t kHeaderBytes = 64 * 1024; // status word at 0, adjoint partial sums at 256
int fail(int code, const char* fmt, ...);
int fail_hip(hipError_t e, const char* what);
size_t align256(size_t v);
int check_dims(const int64_t dims[3], int64_t* n);
int check_eb(float eb);
int check_params(const qai_params* p, qai_params* out);
Tuning tuning_now();
void prof_suppress(bool on);               // pause stage timing on this thread (nests)
uint32_t* word_buffer(void* ws, int64_t cap, int k); // k-th region, cap = word_capacity
void ws_buffers(void* ws, Plan1& p); // status word, the three word buffers and the flags (extents set in p)
int tuning_to_abi(const Tuning& t, qai_tuning* out);
int abi_to_tuning(const qai_tuning* in, Tuning& t); // validates; QAI_EINVAL with a message
Tuning tuning_for(const int64_t dims[3]);           // the setting a plain call on dims uses
void clear_error();
} // namespace api

} // namespace qai
