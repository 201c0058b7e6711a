// qai_code.h -- device-side decoding of the segment code of quantization
// indices (see qai_coded in qai.h): x-rows in segments of 32 voxels, each
// with its first index, the width b of its 31 zigzag-coded differences to the
// prior index, and those differences packed LSB-first in its payload words.
//
// A lane decodes V consecutive indices [p0, p0 + V) of one segment (p0 a
// multiple of V, V dividing 32) in three steps, so that a caller can keep the
// loads of later lines in flight while it works on the current one:
//   code_head   the segment's meta word and first index (two loads);
//   code_words  the payload words that hold the lane's differences (four
//               buffer loads, addressed from the meta word);
//   code_finish the differences' sum, the exclusive prefix over the G = 32 / V
//               lanes of the segment (consecutive lanes of the wave, which must
//               all call it together) and the first index.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qai {

struct CodeHead {
    uint64_t mt;  // (first payload word << 8) | b
    int32_t b0;   // the segment's first index
};

// Payload reads are buffer loads: past the payload they return 0.
constexpr uint32_t kCodeNoRead = 0x80000000u;

__device__ __forceinline__ CodeHead code_head(const int32_t* __restrict__ base, const uint64_t* __restrict__ meta,
                                              int64_t ks)
{
    return CodeHead{meta[ks], base[ks]};
}

// The lane's differences are bits [first, first + V b) of the segment's
// payload, first = (p0 - 1) b (0 for p0 = 0).  Four words hold them when
// b < 32 and (first mod 32) + V b <= 128 ("narrow"); otherwise code_finish
// reads two words per difference itself.
template <int V>
__device__ __forceinline__ bool code_narrow(uint64_t mt)
{
    const uint32_t bw = (uint32_t)(mt & 0xFFu);
    return bw < 32u && bw * V + 31u <= 128u;
}

template <int V>
__device__ __forceinline__ void code_words(__amdgpu_buffer_rsrc_t pay, const CodeHead& h, int p0, uint32_t (&w4)[4])
{
    const uint32_t bw = (uint32_t)(h.mt & 0xFFu);
    const uint32_t wo = (uint32_t)(h.mt >> 8);
    const uint32_t first = (uint32_t)(p0 > 0 ? p0 - 1 : 0) * bw;
    const uint32_t wb = (bw && code_narrow<V>(h.mt)) ? (wo + (first >> 5)) * 4u : kCodeNoRead;
#pragma unroll
    for (int u = 0; u < 4; ++u)
        w4[u] = __builtin_amdgcn_raw_buffer_load_b32(pay, wb == kCodeNoRead ? kCodeNoRead : wb + 4u * u, 0, 0);
}

template <int V>
__device__ __forceinline__ void code_finish(__amdgpu_buffer_rsrc_t pay, const CodeHead& h, const uint32_t (&w4)[4],
                                            int p0, int lane, int32_t (&q)[V])
{
    static_assert(32 % V == 0, "a lane's share lies in one segment");
    constexpr int G = 32 / V;
    const int bw = (int)(h.mt & 0xFFu);
    const uint32_t wo = (uint32_t)(h.mt >> 8);
    const uint64_t mask = (bw >= 32) ? 0xFFFFFFFFull : ((1ull << bw) - 1ull);
    const uint32_t first = (uint32_t)(p0 > 0 ? p0 - 1 : 0) * (uint32_t)bw;
    const bool narrow = code_narrow<V>(h.mt);
    // narrow: the four words as one 128-bit window, shifted right so that the
    // next difference sits at bit 0 (funnel shifts; b < 32)
    const uint32_t f = first & 31u;
    uint32_t r0 = __builtin_amdgcn_alignbit(w4[1], w4[0], f), r1 = __builtin_amdgcn_alignbit(w4[2], w4[1], f);
    uint32_t r2 = __builtin_amdgcn_alignbit(w4[3], w4[2], f), r3 = w4[3] >> f;
    int32_t acc = 0;
#pragma unroll
    for (int j = 0; j < V; ++j) {
        const int i = p0 + j;
        uint32_t zc = 0u;
        if (i > 0) {
            if (narrow) {
                zc = r0 & (uint32_t)mask;
                r0 = __builtin_amdgcn_alignbit(r1, r0, (uint32_t)bw);
                r1 = __builtin_amdgcn_alignbit(r2, r1, (uint32_t)bw);
                r2 = __builtin_amdgcn_alignbit(r3, r2, (uint32_t)bw);
                r3 >>= (uint32_t)bw;
            } else {
                const uint32_t bit = (uint32_t)(i - 1) * (uint32_t)bw;
                const uint32_t wd = (wo + (bit >> 5)) * 4u;
                const uint32_t lo = __builtin_amdgcn_raw_buffer_load_b32(pay, wd, 0, 0);
                const uint32_t hi = __builtin_amdgcn_raw_buffer_load_b32(pay, wd + 4u, 0, 0);
                zc = (uint32_t)(((((uint64_t)hi << 32) | lo) >> (bit & 31u)) & mask);
            }
        }
        acc += (int32_t)((zc >> 1) ^ (0u - (zc & 1u)));
        q[j] = acc;
    }
    int32_t inc = acc;
#pragma unroll
    for (int d = 1; d < G; d <<= 1) {
        const int32_t t = __shfl_up(inc, d, G);
        if ((lane & (G - 1)) >= d)
            inc += t;
    }
    const int32_t b0 = h.b0 + (inc - acc);
#pragma unroll
    for (int j = 0; j < V; ++j)
        q[j] += b0;
}

// The three steps back to back.
template <int V>
__device__ __forceinline__ void decode_share(const int32_t* __restrict__ base, const uint64_t* __restrict__ meta,
                                             __amdgpu_buffer_rsrc_t pay, int64_t ks, int p0, int lane,
                                             int32_t (&q)[V])
{
    const CodeHead h = code_head(base, meta, ks);
    uint32_t w4[4];
    code_words<V>(pay, h, p0, w4);
    code_finish<V>(pay, h, w4, p0, lane, q);
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t payload_rsrc(const uint32_t* p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t*>(p), (short)0, (int)bytes, 0x00020000);
}

} // namespace qai
