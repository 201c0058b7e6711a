// qai_code.h -- device-side decoding of the segment code of quantization
// indices (see qai_coded in qai.h): x-rows in segments of 32 voxels, each
// with its first index, the width b of its 31 zigzag-coded differences to the
// prior index, and those differences packed LSB-first in its payload words.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qai {

// Indices [p0, p0 + V) of segment ks, p0 a multiple of V and V dividing 32:
// the G = 32 / V lanes of a segment are consecutive lanes of the wave and
// must all call this together.  Each lane reads its differences (bits
// [first, first + V b) of the segment's payload: four words hold them when
// (first mod 32) + V b <= 128, else every difference reads its own two
// words), sums them, and adds the exclusive prefix of its lane group to the
// segment's first index.  Payload reads are buffer loads: past the payload
// they return 0.
template <int V>
__device__ __forceinline__ void decode_share(const int32_t* __restrict__ base, const uint64_t* __restrict__ meta,
                                             __amdgpu_buffer_rsrc_t pay, int64_t ks, int p0, int lane,
                                             int32_t (&q)[V])
{
    static_assert(32 % V == 0, "a lane's share lies in one segment");
    constexpr int G = 32 / V;
    const uint64_t mt = meta[ks];
    const int bw = (int)(mt & 0xFFu);
    const uint32_t wo = (uint32_t)(mt >> 8);
    const uint64_t mask = (bw >= 32) ? 0xFFFFFFFFull : ((1ull << bw) - 1ull);
    const uint32_t first = (uint32_t)(p0 > 0 ? p0 - 1 : 0) * (uint32_t)bw;
    const bool narrow = (uint32_t)bw * V + 31u <= 128u;
    const uint32_t wb = bw ? (wo + (first >> 5)) * 4u : 0x80000000u; // width 0: no payload read
    uint32_t w4[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
        w4[u] = __builtin_amdgcn_raw_buffer_load_b32(pay, narrow ? wb + 4u * u : 0x80000000u, 0, 0);
    int32_t acc = 0;
#pragma unroll
    for (int j = 0; j < V; ++j) {
        const int i = p0 + j;
        const uint32_t bit = (uint32_t)(i > 0 ? i - 1 : 0) * (uint32_t)bw;
        uint32_t lo, hi;
        if (narrow) {
            const uint32_t wi = (bit - (first & ~31u)) >> 5;
            lo = wi == 0 ? w4[0] : (wi == 1 ? w4[1] : (wi == 2 ? w4[2] : w4[3]));
            hi = wi == 0 ? w4[1] : (wi == 1 ? w4[2] : w4[3]);
        } else {
            const uint32_t wd = (wo + (bit >> 5)) * 4u;
            lo = __builtin_amdgcn_raw_buffer_load_b32(pay, wd, 0, 0);
            hi = __builtin_amdgcn_raw_buffer_load_b32(pay, wd + 4u, 0, 0);
        }
        const uint32_t zc = (i > 0) ? (uint32_t)(((((uint64_t)hi << 32) | lo) >> (bit & 31u)) & mask) : 0u;
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
    const int32_t b0 = base[ks] + (inc - acc);
#pragma unroll
    for (int j = 0; j < V; ++j)
        q[j] += b0;
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t payload_rsrc(const uint32_t* p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t*>(p), (short)0, (int)bytes, 0x00020000);
}

} // namespace qai
