// Device helpers shared by the library's kernels (query, ordering, training).
#pragma once

#include <hip/hip_runtime.h>

#include "nif_internal.h"

namespace nif {

// ----------------------------------------------------------------------------
// Clip and normalisation, binary32, no contraction.
// Returns 1 if the segment [max(t_near,0), min(t_far,t_max)] is non-empty.
// ----------------------------------------------------------------------------
// The segment alone: true iff [ta, tb] = [max(t_near, 0), min(t_far, t_max)]
// is non-empty (box lo, hi).
__device__ __forceinline__ bool clip_segment(const float o[3], const float d[3], float tmax, const float lo[3],
                                             const float hi[3], float& ta, float& tb) {
#pragma clang fp contract(off)
    float tn = -INFINITY, tf = INFINITY;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0f) {
            if (o[a] < lo[a] || o[a] > hi[a]) return false;
            continue;
        }
        float t0 = (lo[a] - o[a]) / d[a];
        float t1 = (hi[a] - o[a]) / d[a];
        float l = t0 < t1 ? t0 : t1, h = t0 < t1 ? t1 : t0;
        if (l > tn) tn = l;
        if (h < tf) tf = h;
    }
    ta = tn > 0.0f ? tn : 0.0f;
    tb = tf < tmax ? tf : tmax;
    return ta <= tb;
}

// ta, tb receive the segment's ends (also when it is empty).
__device__ __forceinline__ int clip_normalise(const float o[3], const float d[3], float tmax, const ObjDev& b,
                                              float u[3][3], float& ta, float& tb) {
#pragma clang fp contract(off)
    if (!clip_segment(o, d, tmax, b.lo, b.hi, ta, tb)) return 0;
    float len2 = d[0] * d[0];
    len2 = len2 + d[1] * d[1];
    len2 = len2 + d[2] * d[2];
    float len = sqrtf(len2);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float pin = o[a] + ta * d[a];
        float pout = o[a] + tb * d[a];
        float ui = (pin - b.lo[a]) / b.ext[a];
        float uo = (pout - b.lo[a]) / b.ext[a];
        float ud = (d[a] / len + 1.0f) * 0.5f;
        // clamp to [0, 1]; NaN (an infinite segment end) maps to 0
        u[0][a] = ui > 0.0f ? (ui < 1.0f ? ui : 1.0f) : 0.0f;
        u[1][a] = uo > 0.0f ? (uo < 1.0f ? uo : 1.0f) : 0.0f;
        u[2][a] = ud > 0.0f ? (ud < 1.0f ? ud : 1.0f) : 0.0f;
    }
    return 1;
}

__device__ __forceinline__ int clip_normalise(const float o[3], const float d[3], float tmax, const ObjDev& b,
                                              float u[3][3]) {
    float ta, tb;
    return clip_normalise(o, d, tmax, b, u, ta, tb);
}

// Entry point only (the ordering key): same segment test and same entry
// coordinates as clip_normalise.
__device__ __forceinline__ int clip_entry(const float o[3], const float d[3], float tmax, const ObjDev& b,
                                          float uin[3]) {
#pragma clang fp contract(off)
    float ta, tb;
    if (!clip_segment(o, d, tmax, b.lo, b.hi, ta, tb)) return 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float pin = o[a] + ta * d[a];
        float ui = (pin - b.lo[a]) / b.ext[a];
        uin[a] = ui > 0.0f ? (ui < 1.0f ? ui : 1.0f) : 0.0f;
    }
    return 1;
}

__device__ __forceinline__ bool valid_query(const float o[3], const float d[3], float tmax, int32_t id, int32_t K) {
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) ok = ok && isfinite(o[a]) && isfinite(d[a]);
    ok = ok && !(d[0] == 0.0f && d[1] == 0.0f && d[2] == 0.0f);
    ok = ok && !(tmax != tmax) && tmax >= 0.0f;
    ok = ok && id >= 0 && id < K;
    return ok;
}

// Domain-error bits of a query (0 for a valid one): 1 = non-finite origin or
// direction, zero direction, or t_max NaN or negative; 2 = object id out of
// range.
__device__ __forceinline__ uint32_t query_error_bits(const float o[3], const float d[3], float tmax, int32_t id,
                                                     int32_t K) {
    bool ray_ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) ray_ok = ray_ok && isfinite(o[a]) && isfinite(d[a]);
    ray_ok = ray_ok && !(d[0] == 0.0f && d[1] == 0.0f && d[2] == 0.0f);
    ray_ok = ray_ok && !(tmax != tmax) && tmax >= 0.0f;
    return (ray_ok ? 0u : 1u) | (id >= 0 && id < K ? 0u : 2u);
}

}  // namespace nif
