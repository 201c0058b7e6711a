// qai_device.h -- device-side helpers shared by the libqai kernels (gfx950).
//
// Packed distance word.  Every EDT pass moves one 32-bit word per voxel:
//     word = (d2 << 2) | code,   d2 = squared distance to the nearest site,
//     code = sign payload of that site: 0 -> S = 0, 1 -> S = +1, 2 -> S = -1,
// and QAI_WORD_INF (all ones) for "no site on this line/plane/volume yet".
// With extents <= 16384 every real squared distance is <= 3 * 16383^2 <
// 2^30, so a real word never reaches QAI_WORD_INF.  Carrying the sign of the
// chosen site with its distance is what replaces the paper's nearest-boundary
// index I1 and its gather S[I1] (Algorithm 3): each pass keeps, among tied
// sites, the one with the lowest coordinate along its axis, exactly as
// Algorithm 1's strict comparisons do, so the payload is the sign of the
// same boundary voxel I1 designates.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define QAI_WORD_INF 0xFFFFFFFFu
#define QAI_WAVE 64
#define QAI_NUM_XCD 8

namespace qai {

__device__ __forceinline__ uint32_t word_make(uint32_t d2, uint32_t code) { return (d2 << 2) | code; }
__device__ __forceinline__ uint32_t word_d2(uint32_t w) { return w >> 2; }
__device__ __forceinline__ int word_sign(uint32_t w)
{
    // code 1 -> +1, code 2 -> -1, code 0 or no site -> 0
    uint32_t c = (w == QAI_WORD_INF) ? 0u : (w & 3u);
    return c == 1u ? 1 : (c == 2u ? -1 : 0);
}
__device__ __forceinline__ uint32_t sign_code(int s) { return s > 0 ? 1u : (s < 0 ? 2u : 0u); }

// Saturating add of a squared offset (already shifted by 2) to a word: an
// absent site stays absent.
__device__ __forceinline__ uint32_t word_add(uint32_t w, uint32_t add_shifted)
{
    uint32_t r = w + add_shifted;
    return (r < w) ? QAI_WORD_INF : r;
}

// Workgroups are dealt to the 8 XCDs round-robin (workgroup b runs on XCD
// b % 8).  Remap so each XCD receives one contiguous range of logical tiles:
// neighbouring tiles then share that XCD's L2.  A bijection on [0, total).
__device__ __forceinline__ uint64_t xcd_remap(uint64_t b, uint64_t total)
{
    uint64_t xcd = b % QAI_NUM_XCD, local = b / QAI_NUM_XCD;
    uint64_t per = total / QAI_NUM_XCD, rem = total % QAI_NUM_XCD;
    return xcd * per + (xcd < rem ? xcd : rem) + local;
}

// Eq. 1 inverted: q = rintf(x' / (2 eb)) with the IEEE single-precision
// quotient.  The product with the rounded reciprocal differs from the
// correctly rounded quotient by at most 2.5 ulp; for |t| < 2^18 that is below
// 0.04, so whenever the product lies within 0.4 of an integer both round to
// it.  Otherwise (ties, large or non-finite values) the exact division is
// taken.  |q| > 2^21 or a non-finite input sets *bad and yields 0.
__device__ __forceinline__ int32_t recover_q(float x, float inv2eb, float two_eb, bool& bad)
{
    float t = x * inv2eb;
    float r = rintf(t);
    if (fabsf(t) < 262144.0f && fabsf(t - r) <= 0.4f)
        return (int32_t)r;
    float t2 = x / two_eb;
    if (!(fabsf(t2) <= 2097152.0f)) {
        bad = true;
        return 0;
    }
    return (int32_t)rintf(t2);
}

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Workgroup barrier that orders LDS only.  __syncthreads() also orders global
// memory, which on this target waits for every outstanding global load and
// store first: in a loop that prefetches rows from HBM it would wait for the
// prefetch at every barrier.  Kernels whose barriers guard LDS buffers alone
// (no global data passed between waves) use this one.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Highest set bit of m at or below lane (inclusive), or -1.
__device__ __forceinline__ int highest_at_or_below(uint64_t m, int lane)
{
    uint64_t mm = (lane == 63) ? m : (m & ((2ull << lane) - 1ull));
    return mm ? 63 - __clzll(mm) : -1;
}
// Lowest set bit of m at or above lane (inclusive), or -1.
__device__ __forceinline__ int lowest_at_or_above(uint64_t m, int lane)
{
    uint64_t mm = m & (~0ull << lane);
    return mm ? __ffsll((unsigned long long)mm) - 1 : -1;
}

// Interpolation weight of step E in single precision (Section V): the weight
// of the quantization-boundary value for squared distances d1sq to B1 and
// d2sq to B2 (d1_none / d2_none: that boundary set is empty).  Cases in
// order: on B1 -> 1; on B2 -> 0; no B2 anywhere (1/k2 = 0) -> 1; no B1 -> 0;
// otherwise k1^-p / (k1^-p + k2^-p), for p = 1 (1/k1) / (1/k1 + 1/k2).
__device__ __forceinline__ float idw_weight(uint32_t d1sq, bool d1_none, uint32_t d2sq, bool d2_none, float power)
{
    if (!d1_none && d1sq == 0u)
        return 1.0f;
    if (!d2_none && d2sq == 0u)
        return 0.0f;
    if (d2_none)
        return 1.0f;
    if (d1_none)
        return 0.0f;
    float k1 = sqrtf((float)d1sq);
    float k2 = sqrtf((float)d2sq);
    if (power == 1.0f)
        return k2 / (k1 + k2);
    return 1.0f / (1.0f + powf(k1 / k2, power));
}

} // namespace qai
