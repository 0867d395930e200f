// Query ordering for gather locality: a bucket sort of the queries by
// (object, Morton code of the AABB entry point).
//
// The paper groups rays per object only when each object has its own network
// (Sec. 4.1); here grouping by object also keeps every wave on one MLP, and
// ordering by entry point makes the 32 queries of a wave hit neighbouring grid
// cells, so their trilinear gathers share cache lines.  Queries that miss their
// AABB or are invalid go to a last bucket.
//
// Passes: (1) key + rank: each query computes its bucket and takes a rank in it
// with one atomic increment; (2) exclusive scan of the bucket counts (reduce,
// top-level scan, down-sweep); (3) scatter: perm[offset[bucket] + rank] = query.
// The order inside a bucket depends on atomic arrival; the outputs do not,
// because every query is computed independently of its neighbours.
#include "nif_device.h"
#include "nif_internal.h"

namespace nif {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;  // elements per scan block

__device__ __forceinline__ uint32_t spread3(uint32_t v) {
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__global__ void fill_u32_kernel(uint32_t* p, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void order_keys_kernel(OrderArgs A) {
    const uint32_t cells = 1u << A.bits;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < A.n; i += (int64_t)gridDim.x * blockDim.x) {
        const float* r = A.rays + i * 6;
        float o[3] = {r[0], r[1], r[2]}, d[3] = {r[3], r[4], r[5]};
        const float tm = A.tmax[i];
        const int32_t id = A.ids[i];
        uint32_t b = A.num_buckets - 1;
        if (valid_query(o, d, tm, id, A.num_objects)) {
            float u[3][3];
            const ObjDev ob = A.objs[id];
            if (clip_normalise(o, d, tm, ob, u)) {
                uint32_t c[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    uint32_t v = (uint32_t)(u[0][a] * (float)cells);  // u in [0, 1]
                    c[a] = v < cells ? v : cells - 1;
                }
                b = ((uint32_t)id << (3 * A.bits)) | spread3(c[0]) | (spread3(c[1]) << 1) | (spread3(c[2]) << 2);
            }
        }
        A.bucket[i] = b;
        A.rank[i] = atomicAdd(&A.hist[b], 1u);
    }
}

// Sum of the counts of one scan tile.
__global__ __launch_bounds__(kScanThreads) void scan_reduce_kernel(const uint32_t* hist, int64_t n, uint32_t* sums) {
    __shared__ uint32_t ws[kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) s += hist[base + k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kScanThreads / 64; ++w) t += ws[w];
        sums[blockIdx.x] = t;
    }
}

// Exclusive scan of up to kScanThreads * kScanItems tile sums, one block.
__global__ __launch_bounds__(kScanThreads) void scan_top_kernel(uint32_t* sums, int64_t n) {
    __shared__ uint32_t ws[kScanThreads / 64];
    const int64_t base = threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = base + k < n ? sums[base + k] : 0u;
        s += v[k];
    }
    // inclusive scan of per-thread sums across the wave
    const int lane = threadIdx.x & 63;
    uint32_t inc = s;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t t = __shfl_up(inc, off);
        if (lane >= off) inc += t;
    }
    if (lane == 63) ws[threadIdx.x >> 6] = inc;
    __syncthreads();
    uint32_t wave_off = 0;
    for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) wave_off += ws[w];
    uint32_t run = wave_off + inc - s;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) sums[base + k] = run;
        run += v[k];
    }
}

// Exclusive scan of one tile in place, offset by the tile's prefix.
__global__ __launch_bounds__(kScanThreads) void scan_down_kernel(uint32_t* hist, int64_t n, const uint32_t* sums) {
    __shared__ uint32_t ws[kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = base + k < n ? hist[base + k] : 0u;
        s += v[k];
    }
    const int lane = threadIdx.x & 63;
    uint32_t inc = s;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t t = __shfl_up(inc, off);
        if (lane >= off) inc += t;
    }
    if (lane == 63) ws[threadIdx.x >> 6] = inc;
    __syncthreads();
    uint32_t wave_off = 0;
    for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) wave_off += ws[w];
    uint32_t run = sums[blockIdx.x] + wave_off + inc - s;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) hist[base + k] = run;
        run += v[k];
    }
}

__global__ void order_scatter_kernel(OrderArgs A) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < A.n; i += (int64_t)gridDim.x * blockDim.x)
        A.perm[A.hist[A.bucket[i]] + A.rank[i]] = (uint32_t)i;
}

int order_bits(int32_t num_objects) {
    // at most 2^22 buckets in all, at most 2^18 per object
    int bits = 6;
    while (bits > 0 && ((int64_t)num_objects << (3 * bits)) > ((int64_t)1 << 22)) --bits;
    return bits;
}

size_t order_workspace_bytes(int64_t n, int32_t num_objects) {
    const int bits = order_bits(num_objects);
    const int64_t nb = ((int64_t)num_objects << (3 * bits)) + 1;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const int64_t tiles = (nb + kScanTile - 1) / kScanTile;
    return al(nb * 4) + al(tiles * 4) + 3 * al(n * 4);
}

hipError_t launch_order(OrderArgs A, void* ws, hipStream_t s, const uint32_t** perm_out) {
    A.bits = order_bits(A.num_objects);
    const int64_t nb = ((int64_t)A.num_objects << (3 * A.bits)) + 1;
    A.num_buckets = (uint32_t)nb;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const int64_t tiles = (nb + kScanTile - 1) / kScanTile;
    uint8_t* p = reinterpret_cast<uint8_t*>(ws);
    A.hist = reinterpret_cast<uint32_t*>(p);
    p += al(nb * 4);
    A.block_sums = reinterpret_cast<uint32_t*>(p);
    p += al(tiles * 4);
    A.bucket = reinterpret_cast<uint32_t*>(p);
    p += al(A.n * 4);
    A.rank = reinterpret_cast<uint32_t*>(p);
    p += al(A.n * 4);
    if (!A.perm) A.perm = reinterpret_cast<uint32_t*>(p);  // else the caller's buffer
    *perm_out = A.perm;
    if (tiles > kScanTile) return hipErrorInvalidValue;
    const unsigned fb = (unsigned)((nb + 255) / 256 < 4096 ? (nb + 255) / 256 : 4096);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(fb), dim3(256), 0, s, A.hist, nb, 0u);
    const unsigned qb = (unsigned)((A.n + 255) / 256 < 8192 ? (A.n + 255) / 256 : 8192);
    hipLaunchKernelGGL(order_keys_kernel, dim3(qb), dim3(256), 0, s, A);
    hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, A.hist, nb, A.block_sums);
    hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(kScanThreads), 0, s, A.block_sums, tiles);
    hipLaunchKernelGGL(scan_down_kernel, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, A.hist, nb, A.block_sums);
    hipLaunchKernelGGL(order_scatter_kernel, dim3(qb), dim3(256), 0, s, A);
    return hipGetLastError();
}

}  // namespace nif
