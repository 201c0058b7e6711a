/*
 * qai.h -- C ABI of libqai, the MI355X (gfx950) implementation of the
 * quantization-aware interpolation (QAI) decompression post-pass of
 * Jiao et al., "Mitigating Artifacts in Pre-quantization Based Scientific
 * Data Compressors with Quantization-aware Interpolation" (arXiv 2602.20097).
 *
 * The header is HIP-free: device pointers are plain pointers and a stream is
 * a hipStream_t passed as void* (NULL = the null stream).
 *
 * Data layout (every entry point): a field is a dense row-major FP32 array of
 * dims = {nz, ny, nx}, x fastest (the paper's Q[i,j,k] with k innermost,
 * Algorithm 2).  A 2-D field is {1, ny, nx}; a 1-D field {1, 1, nx}.  Each
 * extent must lie in [1, QAI_MAX_EXTENT].
 *
 * Error convention: every entry point returns QAI_OK (0) or a negative code.
 * Argument errors are detected on the host before anything is enqueued.
 * Launch failures return QAI_EHIP; qai_last_error() gives the text (per
 * thread).  Faults inside kernels surface at the caller's next
 * synchronisation, as HIP reports them.  Nothing aborts and nothing throws.
 *
 * Determinism: results are bit-identical across runs, launch shapes and
 * autotuner choices.  Calls are reentrant when their workspaces differ.
 *
 * Streams: a call's work is ordered after what stream holds before it and
 * before what is enqueued on stream after it.  On a 3-D field without taps
 * part of step E runs on a side stream the library keeps per device (created
 * on the device's first call, kept until the process ends), joined to stream
 * with events.  While stream is being captured into a graph, and in
 * qai_mitigate_noalloc, every launch stays on stream.
 */
#ifndef QAI_H
#define QAI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QAI_MAX_EXTENT 16384

enum {
    QAI_OK = 0,
    QAI_EINVAL = -1, /* null pointer, non-finite or non-positive bound/parameter */
    QAI_EDIMS = -2,  /* an extent outside [1, QAI_MAX_EXTENT] */
    QAI_ENOWS = -3,  /* workspace missing or smaller than qai_workspace_bytes() */
    QAI_EHIP = -4,   /* a HIP runtime call or kernel launch failed */
    QAI_ENODEV = -5, /* no usable GPU */
    QAI_ESTATE = -6  /* object used in a state that does not allow the call */
};

/* Device status bits reported by qai_device_status() after a run. */
#define QAI_STATUS_QRANGE 0x1u /* some |x'/(2 eb)| > 2^21 or not finite: output unspecified */

/* Interpolation parameters (Section V, step E).  eta is the boundary
 * magnitude factor (the paper uses 0.9); power is the inverse-distance
 * exponent p of w = k1^-p / (k1^-p + k2^-p) (the paper's weight is p = 1).
 * flags is reserved and must be 0. */
typedef struct {
    float eta;
    float power;
    uint32_t flags;
} qai_params;

/* Optional per-voxel intermediates, each a device array of N = nz*ny*nx
 * entries or NULL:
 *   q     recovered quantization index (Eq. 1)
 *   b1    1 on a quantization boundary B1 (Algorithm 2), else 0
 *   sb    boundary sign S_B in {-1, 0, +1} (Algorithm 2), 0 off B1
 *   s     propagated sign S (Algorithm 3)
 *   d1sq  squared distance to B1 (step B), -1 when B1 is empty
 *   b2    1 on a sign-flipping boundary B2 (Algorithm 3), else 0
 *   d2sq  squared distance to B2 (step D), -1 when B2 is empty
 *   w     interpolation weight in [0, 1] (step E) */
typedef struct {
    int32_t* q;
    uint8_t* b1;
    int8_t* sb;
    int8_t* s;
    int32_t* d1sq;
    uint8_t* b2;
    int32_t* d2sq;
    float* w;
} qai_taps;

/* qai_mitigate -- the whole post-pass, Algorithm 4 (Distance-Based
 * Compensation): out = field + C, C = w * S * eta * eb, with the default
 * parameters eta = 0.9, p = 1.
 *   field  device FP32[N], the decompressed data x' = 2 eb q (Eq. 1); the
 *          indices q are recovered as rintf(field / (2 eb)) and must satisfy
 *          |q| <= 2^21 (else QAI_STATUS_QRANGE is raised, see below)
 *   dims   host int64[3] = {nz, ny, nx}
 *   eb     absolute error bound used by the pre-quantization (> 0, finite)
 *   out    device FP32[N]; may equal field (in place), may not partly overlap
 *   stream hipStream_t or NULL
 * Allocates and frees its workspace stream-ordered (hipMallocAsync); callers
 * that must not allocate use qai_mitigate_ex. */
int qai_mitigate(const float* field, const int64_t dims[3], float eb, float* out, void* stream);

/* Bytes of device workspace qai_mitigate_ex needs for dims: a 64 KiB header
 * (status word, reduction partials), three buffers of 32-bit words (the packed
 * distance words of the passes, ping-ponged), each of nz * ceil(ny/4)*4 * nx
 * words (one per voxel, ny rounded up to a multiple of 4 for a blocked
 * intermediate layout), and one bit per voxel (flags of the fused final pass:
 * 128 bytes per 1024 voxels, rounded up), each part rounded up to 256 bytes.
 * 0 for invalid dims. */
size_t qai_workspace_bytes(const int64_t dims[3]);

/* qai_mitigate_ex -- as qai_mitigate with explicit parameters (NULL = the
 * defaults), a caller-owned device workspace ws of ws_bytes >=
 * qai_workspace_bytes(dims) (any alignment of 256 bytes or more), and optional
 * taps (NULL = none).  Afterwards the workspace holds the final distance word
 * of the first EDT at every voxel, and the final word of the second EDT at
 * every voxel whose weight depends on it (S != 0 and not on B1), which is all
 * qai_backward reads; keep the workspace untouched until then.  On a 3-D field
 * without taps, with default pass choices and 16-byte aligned field and out,
 * and on a 2-D field without taps whose y pass of the second EDT is on
 * automatic or the direct search (edt2_algo[0] -1 or 5), the second EDT's last
 * pass runs only at those voxels, so its words elsewhere are left unspecified;
 * every other call writes them at every voxel. */
int qai_mitigate_ex(const float* field, const int64_t dims[3], float eb, const qai_params* params,
                    void* ws, size_t ws_bytes, float* out, const qai_taps* taps, void* stream);

/* qai_backward -- adjoint of step E (project addition, not in the paper).
 * The EDTs are piecewise constant in the data and are held fixed, so
 *   d out / d field = identity            (grad_field = grad_out, not written)
 *   dL/d eta   = sum_i g_i * w_i * S_i * eb
 *   dL/d power = sum_i g_i * S_i * eta * eb * (-w_i (1 - w_i) ln(k1_i / k2_i))
 * (0 wherever w is pinned at 0 or 1).
 *   grad_out     device FP32[N], dL/d out
 *   ws_saved     the workspace of the qai_mitigate_ex call being
 *                differentiated (same dims); its header is reused for the
 *                partial sums
 *   grad_params  device FP32[2] receiving {dL/d eta, dL/d power} (overwritten)
 * The reduction is deterministic (fixed tree, FP64 partial sums). */
int qai_backward(const float* grad_out, void* ws_saved, size_t ws_bytes, const int64_t dims[3],
                 float eb, const qai_params* params, float* grad_params, void* stream);

/* qai_mitigate_noalloc -- for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  The same post-pass and result as qai_mitigate_ex with
 * taps = NULL, but the workspace is a fixed device array inside the library of
 * QAI_NOALLOC_SCRATCH_BYTES (256 MiB) on each GPU it runs on, held until the
 * process ends; nothing is allocated or freed.
 *   field, dims, eb, out, stream  as for qai_mitigate
 *   params                        as for qai_mitigate_ex (NULL = defaults)
 * Fields whose qai_workspace_bytes(dims) exceeds QAI_NOALLOC_SCRATCH_BYTES
 * (about 22 million voxels) are rejected with QAI_ENOWS before anything is
 * enqueued.  Every call on one GPU shares that GPU's array, which keeps the
 * last call's contents (each call clears the words it needs cleared with a
 * kernel): calls that overlap on one GPU, on different streams or threads,
 * race and must be serialised by the caller.  The status words live in that
 * array too, so qai_device_status does not apply to these calls. */
#define QAI_NOALLOC_SCRATCH_BYTES (256u << 20)
int qai_mitigate_noalloc(const float* field, const int64_t dims[3], float eb, const qai_params* params, float* out,
                         void* stream);

/* qai_device_status -- synchronises stream and reports the status bits the
 * last run on workspace ws raised (QAI_STATUS_*). */
int qai_device_status(const void* ws, void* stream, uint32_t* flags);

/* Text of the last error on the calling thread ("" if none). */
const char* qai_last_error(void);

/* ------------------------------------------------------------------ batch
 * Batched form (project addition, not in the paper): many fields of uneven
 * shapes processed by one hipGraph launch.  Each field runs the plain
 * pipeline on its own slice of the workspace; fields are dealt, largest
 * first, to up to four independent branches of the graph, so kernels of
 * different fields overlap.  Each field's result is bit-identical to
 * qai_mitigate_ex on it alone. */
typedef struct qai_batch_plan qai_batch_plan;

/* Plan flag: every distinct shape runs its autotuned setting (see
 * qai_autotune): the cached one, or one timed before capture on the first
 * field of that shape (and then cached). */
#define QAI_BATCH_AUTOTUNE 0x1u
/* Plan flag (implies QAI_BATCH_AUTOTUNE): each field then also times the
 * pass-algorithm variants of its shape's setting (first and second EDT:
 * automatic, envelope, windowed) on itself and keeps the fastest, since the
 * best pass choice follows a field's boundary density more than its shape. */
#define QAI_BATCH_TUNE_EACH 0x2u

/* Bytes of device workspace a batch of n fields needs: the sum over fields
 * of qai_workspace_bytes, each rounded up to 256.  0 for invalid input. */
size_t qai_batch_workspace_bytes(int n, const int64_t (*dims)[3]);

/* Build a plan and capture it into a graph.
 *   fields, outs  arrays of n device FP32 pointers (an output may not overlap
 *                 its input)
 *   dims, ebs     n host triples {nz, ny, nx} and n host error bounds
 *   params        shared step-E parameters (NULL = defaults)
 *   flags         0, QAI_BATCH_AUTOTUNE or QAI_BATCH_TUNE_EACH (autotuning runs the pipeline on
 *                 the first field of each shape, writing its output)
 *   ws, ws_bytes  device workspace of qai_batch_workspace_bytes, 256-aligned
 *   stream        stream for the autotuning runs; synchronised before capture
 * The plan keeps the raw pointers until qai_batch_plan_destroy; the settings
 * are fixed at creation (qai_tuning_set afterwards does not change them). */
int qai_batch_plan_create(int n, const float* const* fields, const int64_t (*dims)[3], const float* ebs,
                          float* const* outs, const qai_params* params, uint32_t flags, void* ws, size_t ws_bytes,
                          void* stream, qai_batch_plan** plan);

/* Replay the captured graph on stream (hipGraphLaunch). */
int qai_batch_plan_launch(qai_batch_plan* plan, void* stream);

/* Run the same batch without the graph, one launch per stage per field, in
 * field order on stream (the reference point the graph is compared with). */
int qai_batch_plan_launch_per_field(qai_batch_plan* plan, void* stream);

/* The launch setting the plan uses for field (after autotuning). */
typedef struct qai_tuning qai_tuning;
int qai_batch_plan_tuning(const qai_batch_plan* plan, int field, qai_tuning* t);

void qai_batch_plan_destroy(qai_batch_plan* plan);

/* ------------------------------------------------------------ tuning
 * Launch geometry and per-pass algorithm choice (process-wide; the batched
 * plan captures the setting current at its creation).  Results do not depend
 * on it: every choice computes the same exact transforms. */
typedef struct qai_tuning {
    int32_t edt1_algo[2];  /* y and z passes of the first EDT: 0 streaming envelope, 1 windowed
                              search over LDS tiles, 2 banded envelope over LDS tiles,
                              4 streaming outward search (short distances), 5 outward search
                              per voxel from the pass input (short distances, any number
                              of column tiles); -1 (the default)
                              picks per pass: 5 for the y pass of a 2-D field, else 1 when
                              the pass has fewer than 4096 tiles of 64 columns, else 4; on a
                              3-D field with both passes at -1 they
                              run as one search over (y, z) offsets, with the separable passes
                              (chosen as for -1) behind it where that search does not apply */
    int32_t edt2_algo[2];  /* the same for the second EDT, plus 3: per-lane online envelope
                              (payload-free words; falls back to 0 where its packed ring
                              entries would not fit 32 bits); -1 (the default) picks 5 for
                              the y pass of a 2-D field, else 1 below 256 tiles, else 3.  For the z pass of a 3-D call without taps
                              (16-byte aligned field and out), -1 computes the distance to B2
                              only where step E needs it, by an exact outward search along z
                              fused with step E; an explicit choice runs the whole pass.
                              The y pass of a 2-D call without taps at -1 or 5 runs the
                              direct search only where step E needs it, fused with step E */
    int32_t edt1_ring;     /* live-window ring entries of the streaming envelope: 16, 32 or 64 */
    int32_t edt2_ring;
    int32_t tile_log2[2];  /* log2 of x-columns per tile of the tiled variants, y and z (-1: auto) */
    int32_t seed_rows;     /* x-lines (wavefronts) per workgroup of the LDS-slab seed passes
                              (1..8); 0 selects the register-resident variant (a wave per
                              line of up to 512 voxels, two, four or eight waves per line of
                              up to 1024, 2048 or 4096) wherever x-lines hold at most 4096
                              voxels; -1 the line-per-wave variant (neighbour lines read
                              through the caches) */
    int32_t seed_planes;   /* z-planes marched per workgroup of the seed passes (>= 1) */
    int32_t window_threads; /* threads per workgroup of the windowed variant (64..1024) */
    int32_t force_wide;    /* 0 (the default): each kernel picks 32-bit buffer offsets and 32-bit
                              arithmetic where the field's size allows them; 1: take the 64-bit
                              index and 64-bit arithmetic variants wherever a kernel has one (same
                              results; lets small fields exercise the paths large ones take) */
} qai_tuning;

/* Copy the current setting into *t. */
int qai_tuning_get(qai_tuning* t);
/* Replace the current setting (validated; QAI_EINVAL if out of range).  NULL
 * restores the built-in defaults. */
int qai_tuning_set(const qai_tuning* t);

/* ------------------------------------------------------------ autotuning
 * Project addition.  qai_autotune times candidate settings on one field: the
 * pass algorithms of both EDTs with the seed variants, then, for the fastest,
 * the line-tile shapes (tile_log2) and workgroup sizes (window_threads) of the
 * passes it runs as the windowed search.  The winner is stored in a per-shape
 * cache held by the library; qai_mitigate, qai_mitigate_ex,
 * qai_mitigate_noalloc and batch plans use a shape's cached setting while the
 * process-wide setting is the built-in default (never set, or reset with
 * qai_tuning_set(NULL)).  Results never depend on the setting.
 *   field, dims, eb  as for qai_mitigate_ex
 *   ws, ws_bytes     workspace of qai_workspace_bytes(dims), 256-byte aligned
 *   out              device FP32[N], apart from field (written many times)
 *   best             receives the chosen setting (nullable)
 * Synchronises stream (the candidates are timed with HIP events on it). */
int qai_autotune(const float* field, const int64_t dims[3], float eb, void* ws, size_t ws_bytes, float* out,
                 void* stream, qai_tuning* best);

/* The cache as a text file: a header line, then one line per shape with
 * nz ny nx and the fields of qai_tuning in declaration order (force_wide
 * excluded).  save writes every entry; load validates every line as
 * qai_tuning_set does and adds (or replaces) the entries; QAI_EINVAL on I/O or
 * format errors (nothing is added then). */
int qai_tuning_cache_save(const char* path);
int qai_tuning_cache_load(const char* path);
int qai_tuning_cache_clear(void);
/* Number of shapes in the cache. */
int qai_tuning_cache_size(void);

/* ------------------------------------------------------------ blocks
 * The paper's block-decomposed strategies (Section VI-B) on one GPU.  The
 * field is cut into blocks[0] x blocks[1] x blocks[2] blocks along z, y, x
 * (extents split as evenly as possible, the first blocks one voxel longer),
 * each processed as a field of its own:
 *   QAI_BLOCKS_EP      embarrassingly parallel: each block runs the whole
 *                      post-pass alone (its faces are domain edges);
 *   QAI_BLOCKS_APPROX  approximate: each block sees one ghost layer of its
 *                      neighbours, exchanged twice -- the data for the
 *                      boundary stencil of step A, then the propagated signs
 *                      of step B for the sign-flip stencil of step C -- while
 *                      both EDTs stay local to the block.
 * The exact strategy is qai_mitigate_ex on the whole field.
 *   field, dims, eb, params, out, stream  as for qai_mitigate_ex (no taps)
 *   blocks   host int32[3], each in [1, extent]; at most 4096 blocks
 *   ws       device workspace of qai_blocks_workspace_bytes, 256-aligned:
 *            per block a copy of its (ghosted) region, its output and a
 *            plain workspace; for QAI_BLOCKS_APPROX one word per voxel more
 * A block grid of 1 x 1 x 1 gives qai_mitigate_ex's result. */
#define QAI_BLOCKS_EP 0
#define QAI_BLOCKS_APPROX 1
size_t qai_blocks_workspace_bytes(const int64_t dims[3], const int32_t blocks[3], int mode);
int qai_mitigate_blocks(const float* field, const int64_t dims[3], float eb, const qai_params* params,
                        const int32_t blocks[3], int mode, void* ws, size_t ws_bytes, float* out, void* stream);

/* ------------------------------------------------------------ coded input
 * The post-pass straight from coded quantization indices, with no
 * decompressed copy of the field stored apart from the result.  The code is a
 * simple one of the paper's kind (Section III-A: the indices are predicted and
 * encoded losslessly; cuSZp predicts from one prior value with fixed-length
 * codes): each x-row is cut into segments of 32 voxels (the last one padded
 * by repeating the row's last index); segment k holds base[k] (its first
 * index), meta[k] = (first payload word << 8) | b, and its 31 differences to
 * the prior index, zigzag-coded ((d << 1) ^ (d >> 31)), b bits each (0..32),
 * packed LSB-first from bit 0 of its payload words.  Segments are numbered
 * row by row (ceil(nx / 32) per row).  The payload must hold one word more
 * than the last segment needs.  Offsets are not checked against the payload:
 * words past its end read as 0 (a malformed code gives wrong values, never a
 * fault). */
typedef struct {
    const int32_t* base;     /* device int32[n_seg] */
    const uint64_t* meta;    /* device uint64[n_seg] */
    const uint32_t* payload; /* device uint32[payload_words] */
    uint64_t payload_words;  /* in [1, 2^29) */
    int32_t seg_len;         /* 32 */
} qai_coded;

/* x' = 2 eb q of every voxel (FP32: the exact product rounded once) into the
 * device FP32[N] array xq. */
int qai_decode(const qai_coded* code, const int64_t dims[3], float eb, float* xq, void* stream);

/* qai_mitigate_ex from coded indices (no taps): out receives the result; the
 * first seed pass decodes the indices it reads (lines of up to 512 voxels with
 * ceil(nx / 64) in {1, 2, 4, 8}, and lines of 513 to 2048 voxels; other shapes
 * decode into out first) and writes
 * x' into out, which the later stages read in place.  ws as for
 * qai_mitigate_ex; results equal qai_mitigate_ex on the decoded field. */
int qai_mitigate_coded(const qai_coded* code, const int64_t dims[3], float eb, const qai_params* params, void* ws,
                       size_t ws_bytes, float* out, void* stream);

/* ------------------------------------------------------------ quality
 * The paper's quality metrics (Section III-C), comparing an original field
 * with a decompressed or compensated one on the GPU:
 *   SSIM (Eq. 3): per window, (2 mu1 mu2 + c1)(2 s12 + c2) /
 *     ((mu1^2 + mu2^2 + c1)(s1^2 + s2^2 + c2)) with sample means, sample
 *     variances and covariance (divisor m - 1 for m voxels), c1 = 1e-4,
 *     c2 = 9e-4, both fields normalised by the original's range; windows of 7
 *     voxels per axis (the whole extent on an axis shorter than 7) at a stride
 *     of 2, only whole windows; the result is the mean over windows;
 *   PSNR (Eq. 4): 20 log10((max - min of the original) / sqrt(MSE)).
 *   orig, dec  device FP32[N] of the same dims
 *   ws         device workspace of qai_quality_workspace_bytes(dims), 256-aligned
 *   result     device double[4] receiving {SSIM, PSNR, MSE, value range of orig};
 *              SSIM is NaN for a constant original, PSNR +inf for equal fields
 * QAI_EDIMS when a window would hold fewer than two voxels.  Sums are FP64 in a
 * fixed order: the result is deterministic. */
size_t qai_quality_workspace_bytes(const int64_t dims[3]);
int qai_quality(const float* orig, const float* dec, const int64_t dims[3], void* ws, size_t ws_bytes,
                double* result, void* stream);

/* ------------------------------------------------------------ utilities */

/* Plain device copy of n 32-bit words (a bandwidth probe: the achievable HBM
 * rate that the post-pass is compared with). */
int qai_copy_probe(const void* src, void* dst, size_t n_words, void* stream);

/* Per-stage timing of qai_mitigate_ex calls: when enabled, every call records
 * HIP events around each kernel on the caller's stream; qai_stage_times()
 * synchronises, adds the elapsed milliseconds of each stage since the last
 * reset into ms[0..n-1] and reports the stage count. names (nullable) receives
 * static strings. */
int qai_profile_enable(int on);
int qai_stage_times(double* ms, const char** names, int n, int* n_stages, int reset);

#ifdef __cplusplus
}
#endif

#endif /* QAI_H */
