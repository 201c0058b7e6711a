// qai_codec.hip -- the post-pass straight from coded quantization indices.
//
// The indices of a pre-quantized field (Eq. 1) are coded per x-row in
// segments of 32 voxels: the first index, the width of the 31 differences to
// the prior value (zigzag-coded) and those differences packed LSB-first in the
// segment's own payload words -- the prediction from one prior value and the
// fixed-length code the paper names for cuSZp (Section III-A).
// qai_mitigate_coded feeds the code to the first seed pass, which decodes each
// line it reads and writes the decompressed values x' = 2 eb q into out; every
// later stage takes out as its x', so no decompressed copy of the field is
// ever stored apart from the result.  Lines whose lanes would straddle
// segments take a separate decode (k_decode) into out first.
#include "qai.h"
#include "qai_code.h"
#include "qai_device.h"
#include "qai_kernels.h"

using namespace qai::api;

namespace qai {
namespace {

// Sixteen segments per wave: four lanes per segment, eight voxels per lane
// (decode_share), written as two 16-byte stores where the row allows.
__global__ __launch_bounds__(256) void k_decode(const int32_t* __restrict__ base, const uint64_t* __restrict__ meta,
                                                const uint32_t* __restrict__ pay, uint32_t pay_bytes, int64_t nrows,
                                                int64_t nx, int64_t segs_row, float two_eb, float* __restrict__ xq)
{
    const __amdgpu_buffer_rsrc_t rs = payload_rsrc(pay, pay_bytes);
    const int64_t nseg = nrows * segs_row;
    const int lane = threadIdx.x & 63;
    const int part = lane & 3;
    const int64_t groups = (nseg + 15) / 16; // 16 segments per wave
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; w < groups; w += nwaves) {
        const int64_t k = min(w * 16 + (lane >> 2), nseg - 1); // the last wave repeats the last segment
        int32_t q[8];
        decode_share<8>(base, meta, rs, k, part * 8, lane, q);
        const int64_t row = k / segs_row, sg = k - row * segs_row;
        const int64_t x = sg * 32 + part * 8;
        float* const dst = xq + row * nx + x;
        if (x + 8 <= nx && ((row * nx + x) & 3) == 0 && (((uintptr_t)xq) & 15) == 0) {
            *reinterpret_cast<float4*>(dst) =
                make_float4((float)q[0] * two_eb, (float)q[1] * two_eb, (float)q[2] * two_eb, (float)q[3] * two_eb);
            *reinterpret_cast<float4*>(dst + 4) =
                make_float4((float)q[4] * two_eb, (float)q[5] * two_eb, (float)q[6] * two_eb, (float)q[7] * two_eb);
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (x + j < nx)
                    dst[j] = (float)q[j] * two_eb;
        }
    }
}

int check_code(const qai_coded* c, const int64_t dims[3])
{
    if (!c || !c->base || !c->meta || !c->payload)
        return fail(QAI_EINVAL, "code and its three arrays must not be NULL");
    if (c->seg_len != 32)
        return fail(QAI_EINVAL, "segment length %d: only 32 is supported", c->seg_len);
    if (c->payload_words < 1 || c->payload_words > 0x1FFFFFFFull)
        return fail(QAI_EINVAL, "payload of %llu words outside [1, 2^29)", (unsigned long long)c->payload_words);
    (void)dims;
    return QAI_OK;
}

} // namespace

hipError_t launch_decode(const Coded& c, int64_t nz, int64_t ny, int64_t nx, float two_eb, float* xq, hipStream_t s)
{
    const int64_t segs_row = (nx + 31) / 32, nseg = nz * ny * segs_row;
    const int64_t blocks = (nseg + 63) / 64; // 4 waves of 16 segments
    return launch_checked(k_decode, dim3((uint32_t)(blocks < (1 << 20) ? blocks : (1 << 20))), dim3(256), 0, s,
                          c.base, c.meta, c.payload, (uint32_t)(c.payload_words * 4), nz * ny, nx, segs_row, two_eb,
                          xq);
}

} // namespace qai

extern "C" {

int qai_decode(const qai_coded* code, const int64_t dims[3], float eb, float* xq, void* stream)
{
    clear_error();
    int64_t n;
    int rc = check_dims(dims, &n);
    if (rc)
        return rc;
    if ((rc = qai::check_code(code, dims)))
        return rc;
    if ((rc = check_eb(eb)))
        return rc;
    if (!xq)
        return fail(QAI_EINVAL, "xq must be a device pointer");
    const qai::Coded c = {code->base, code->meta, code->payload, code->payload_words};
    const hipError_t e = qai::launch_decode(c, dims[0], dims[1], dims[2], 2.0f * eb, xq, (hipStream_t)stream);
    return e == hipSuccess ? QAI_OK : fail_hip(e, "decode launch");
}

int qai_mitigate_coded(const qai_coded* code, const int64_t dims[3], float eb, const qai_params* params, void* ws,
                       size_t ws_bytes, float* out, void* stream)
{
    clear_error();
    int64_t n;
    int rc = check_dims(dims, &n);
    if (rc)
        return rc;
    if ((rc = qai::check_code(code, dims)))
        return rc;
    if (!out)
        return fail(QAI_EINVAL, "out must be a device pointer");
    if ((rc = check_eb(eb)))
        return rc;
    qai_params p;
    if ((rc = check_params(params, &p)))
        return rc;
    const size_t need = qai_workspace_bytes(dims);
    if (!ws || ws_bytes < need)
        return fail(QAI_ENOWS, "workspace of %zu bytes needed, %zu given", need, ws ? ws_bytes : (size_t)0);
    if (((uintptr_t)ws & 255u) != 0)
        return fail(QAI_ENOWS, "workspace must be 256-byte aligned");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fail(QAI_ENODEV, "no usable GPU: %s", hipGetErrorString(e));
    const qai::Coded c = {code->base, code->meta, code->payload, code->payload_words};
    qai::Plan1 pl = {};
    pl.coded = &c;
    pl.xq = out;
    pl.out = out;
    pl.nz = dims[0];
    pl.ny = dims[1];
    pl.nx = dims[2];
    pl.eb = eb;
    pl.eta = p.eta;
    pl.power = p.power;
    ws_buffers(ws, pl);
    std::unique_lock<std::mutex> lk;
    if (!qai::stream_capturing((hipStream_t)stream)) {
        if ((e = qai::aux_for(dev, pl.aux)) != hipSuccess)
            return fail_hip(e, "side stream");
        lk = std::unique_lock<std::mutex>(pl.aux->mu);
    }
    e = qai::run_plain(pl, tuning_for(dims), (hipStream_t)stream);
    return e == hipSuccess ? QAI_OK : fail_hip(e, "kernel launch");
}

} // extern "C"
