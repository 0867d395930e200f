// Pair expansion and per-ray combination for scenes of several objects.
//
// The method issues one neural query per (ray, object) pair whose segment
// meets the object's AABB; a ray is visible iff every such pair is visible,
// and a ray that meets no AABB is visible (Sec. 4.1).  The expansion uses the
// same binary32 segment test as the query kernel, so a pair is emitted iff the
// query would not report a miss.
//
// Passes: (1) count the pairs of every ray; (2) exclusive scan of the counts;
// (3) write the pairs in ray order, objects ascending within a ray, and the
// total.
#include "nif_device.h"
#include "nif_internal.h"

namespace nif {

constexpr int kPairThreads = 256;

// Conservative rejection before the exact test: slab distances with a
// reciprocal multiply instead of a division (within 2.5 ulp of the quotient)
// and the interval widened by 8 ulp on each side, so a box the exact binary32
// test accepts is never rejected here.  rcp(d) is only used for |d| >= 2^-100.
struct RayPre {
    float o[3], d[3], inv[3], tm;
    bool fast;
};

__device__ __forceinline__ RayPre ray_pre(const float o[3], const float d[3], float tm) {
    RayPre r;
    r.fast = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        r.o[a] = o[a];
        r.d[a] = d[a];
        r.inv[a] = __builtin_amdgcn_rcpf(d[a]);
        r.fast = r.fast && (d[a] == 0.0f || fabsf(d[a]) >= 0x1p-100f);
    }
    r.tm = tm;
    return r;
}

__device__ __forceinline__ bool maybe_hit(const RayPre& r, const float lo[3], const float hi[3]) {
#pragma clang fp contract(off)
    if (!r.fast) return true;
    constexpr float kWiden = 8.0f * 0x1p-24f;
    float tn = -INFINITY, tf = INFINITY;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (r.d[a] == 0.0f) {
            if (r.o[a] < lo[a] || r.o[a] > hi[a]) return false;
            continue;
        }
        const float t0 = (lo[a] - r.o[a]) * r.inv[a];
        const float t1 = (hi[a] - r.o[a]) * r.inv[a];
        float l = fminf(t0, t1), h = fmaxf(t0, t1);
        l -= kWiden * fabsf(l);
        h += kWiden * fabsf(h);
        tn = fmaxf(tn, l);
        tf = fminf(tf, h);
    }
    const float ta = fmaxf(tn, 0.0f), tb = fminf(tf, r.tm);
    return ta <= tb;
}

// With at most 64 objects the count pass also keeps every ray's hit mask, and
// the emit pass reads it instead of testing the boxes again.
__global__ __launch_bounds__(kPairThreads) void pairs_count_kernel(const float* __restrict__ rays,
                                                                   const float* __restrict__ tmax, int64_t n,
                                                                   const ObjDev* __restrict__ objs, int32_t K,
                                                                   const BoxGroup* __restrict__ groups, int32_t G,
                                                                   uint32_t* __restrict__ counts,
                                                                   uint64_t* __restrict__ masks) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        float o[3], d[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            o[a] = rays[r * 6 + a];
            d[a] = rays[r * 6 + 3 + a];
        }
        const float tm = tmax[r];
        uint32_t c = 0;
        const bool ok = !(query_error_bits(o, d, tm, 0, 1) & 1u);  // invalid rays have no pairs
        const RayPre pre = ray_pre(o, d, tm);
        uint64_t mk = 0;
        if (G > 0) {  // groups first: a box in a group lies inside the group's box
            for (int32_t g = 0; ok && g < G; ++g) {
                if (!maybe_hit(pre, groups[g].lo, groups[g].hi)) continue;
                uint64_t mem = groups[g].members;
                while (mem) {
                    const int k = __builtin_ctzll(mem);
                    mem &= mem - 1;
                    float ta, tb;
                    if (maybe_hit(pre, objs[k].lo, objs[k].hi) &&
                        clip_segment(o, d, tm, objs[k].lo, objs[k].hi, ta, tb)) {
                        ++c;
                        mk |= 1ull << k;
                    }
                }
            }
        } else {
            for (int32_t k = 0; ok && k < K; ++k) {
                float ta, tb;
                if (maybe_hit(pre, objs[k].lo, objs[k].hi) && clip_segment(o, d, tm, objs[k].lo, objs[k].hi, ta, tb)) {
                    ++c;
                    if (k < 64) mk |= 1ull << k;
                }
            }
        }
        counts[r] = c;
        if (masks) masks[r] = mk;
    }
}

__global__ __launch_bounds__(kPairThreads) void pairs_emit_kernel(const float* __restrict__ rays,
                                                                  const float* __restrict__ tmax, int64_t n,
                                                                  const ObjDev* __restrict__ objs, int32_t K,
                                                                  const uint32_t* __restrict__ offsets,
                                                                  int64_t max_pairs, float* __restrict__ pair_rays,
                                                                  float* __restrict__ pair_tmax,
                                                                  int32_t* __restrict__ pair_ids,
                                                                  uint32_t* __restrict__ pair_ray,
                                                                  const uint64_t* __restrict__ masks,
                                                                  int64_t* __restrict__ total) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        float o[3], d[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            o[a] = rays[r * 6 + a];
            d[a] = rays[r * 6 + 3 + a];
        }
        const float tm = tmax[r];
        int64_t p = offsets[r];
        const bool ok = !(query_error_bits(o, d, tm, 0, 1) & 1u);
        const RayPre pre = ray_pre(o, d, tm);
        uint64_t mk = masks ? masks[r] : 0;
        for (int32_t k = 0; ok && k < K; ++k) {
            if (masks) {  // ascending set bits of the stored mask
                if (!mk) break;
                k = __builtin_ctzll(mk);
                mk &= mk - 1;
            } else {
                float ta, tb;
                if (!maybe_hit(pre, objs[k].lo, objs[k].hi) || !clip_segment(o, d, tm, objs[k].lo, objs[k].hi, ta, tb))
                    continue;
            }
            if (p < max_pairs) {
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    pair_rays[p * 6 + a] = o[a];
                    pair_rays[p * 6 + 3 + a] = d[a];
                }
                pair_tmax[p] = tm;
                pair_ids[p] = k;
                pair_ray[p] = (uint32_t)r;
            }
            ++p;
        }
        if (r == n - 1) *total = p;  // offsets are exclusive: the last ray's end is the total
    }
}

__global__ void pairs_zero_total_kernel(int64_t* total) {
    if (threadIdx.x == 0) *total = 0;
}

// Ray visibility: 1 unless some pair of the ray has visibility < 0.5.
__global__ void combine_init_kernel(uint8_t* ray_visible, int64_t n_rays) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n_rays; r += (int64_t)gridDim.x * blockDim.x)
        ray_visible[r] = 1;
}

__global__ void combine_pairs_kernel(const uint32_t* __restrict__ pair_ray, const float* __restrict__ vis,
                                     int64_t n_pairs, int64_t n_rays, uint8_t* __restrict__ ray_visible) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n_pairs; p += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t r = pair_ray[p];
        if (vis[p] < 0.5f && r < n_rays) ray_visible[r] = 0;  // every writer stores the same value
    }
}

size_t pairs_workspace_bytes(int64_t n_rays, int32_t K) {
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    return al((size_t)n_rays * 4) + al((size_t)scan_block_sums(n_rays) * 4) + (K <= 64 ? al((size_t)n_rays * 8) : 0);
}

static unsigned grid_for(int64_t n, int threads) {
    const int64_t b = (n + threads - 1) / threads;
    return (unsigned)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

hipError_t launch_expand_pairs(const float* rays, const float* tmax, int64_t n, const ObjDev* objs, int32_t K,
                               const BoxGroup* groups, int32_t num_groups, int64_t max_pairs, float* pair_rays, float* pair_tmax, int32_t* pair_ids,
                               uint32_t* pair_ray, int64_t* total, void* ws, hipStream_t s) {
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    uint32_t* counts = reinterpret_cast<uint32_t*>(ws);
    uint32_t* sums = reinterpret_cast<uint32_t*>(reinterpret_cast<uint8_t*>(ws) + al((size_t)n * 4));
    uint64_t* masks = K <= 64 ? reinterpret_cast<uint64_t*>(reinterpret_cast<uint8_t*>(ws) + al((size_t)n * 4) +
                                                          al((size_t)scan_block_sums(n) * 4))
                              : nullptr;
    hipLaunchKernelGGL(pairs_zero_total_kernel, dim3(1), dim3(64), 0, s, total);
    if (n == 0) return hipGetLastError();
    hipLaunchKernelGGL(pairs_count_kernel, dim3(grid_for(n, kPairThreads)), dim3(kPairThreads), 0, s, rays, tmax, n,
                       objs, K, K <= 64 ? groups : nullptr, K <= 64 ? num_groups : 0, counts, masks);
    hipError_t e = launch_exclusive_scan_u32(counts, n, sums, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(pairs_emit_kernel, dim3(grid_for(n, kPairThreads)), dim3(kPairThreads), 0, s, rays, tmax, n,
                       objs, K, counts, max_pairs, pair_rays, pair_tmax, pair_ids, pair_ray, masks, total);
    return hipGetLastError();
}

hipError_t launch_combine_pairs(const uint32_t* pair_ray, const float* vis, int64_t n_pairs, int64_t n_rays,
                                uint8_t* ray_visible, hipStream_t s) {
    if (n_rays > 0)
        hipLaunchKernelGGL(combine_init_kernel, dim3(grid_for(n_rays, 256)), dim3(256), 0, s, ray_visible, n_rays);
    if (n_pairs > 0)
        hipLaunchKernelGGL(combine_pairs_kernel, dim3(grid_for(n_pairs, 256)), dim3(256), 0, s, pair_ray, vis, n_pairs,
                           n_rays, ray_visible);
    return hipGetLastError();
}

}  // namespace nif
