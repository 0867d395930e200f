// Query ordering for gather locality: a bucket sort of the queries by
// (object, Morton code of the AABB entry point).
//
// The paper groups rays per object only when each object has its own network
// (Sec. 4.1); here grouping by object also keeps every wave on one MLP, and
// ordering by entry point makes the 32 queries of a wave hit neighbouring grid
// cells, so their trilinear gathers share cache lines.  Queries that miss their
// AABB or are invalid go to a last bucket.
//
// Passes (no global atomics): (1) each block counts the buckets of its tile of
// queries in LDS and writes them as one row of a (tile x bucket) table;
// (2) per bucket, exclusive scan over the tiles and the bucket's total;
// (3) each block scans the bucket totals into bucket offsets, ranks its
// queries inside (bucket, tile) with LDS counters and scatters
// perm[bucket offset + tile offset + rank] = query.
// The order inside a (bucket, tile) cell depends on LDS atomic arrival;
// (4) optionally, every window of 4096 consecutive entries is then sorted by a
// finer key (8 Morton bits per axis) in LDS, so that a wave's 32 queries cover
// a few finest-level cells (ties keep the bucket order).  The outputs do not
// depend on the order, because every query is computed independently of its
// neighbours.

#include "nif_device.h"
#include "nif_order_key.h"
#include "nif_internal.h"

namespace nif {

__global__ void fill_u32_kernel(uint32_t* p, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t b = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)b), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// Bucket (object, coarse Morton code) of query i; *fine receives the finer key
// (object, Morton code with fine_bits per axis), 0xffffffff for a miss.  The
// coarse code is a prefix of the fine one, so ordering by the fine key refines
// the bucket order.
struct QueryIn {
    float o[3], d[3], tm;
    int32_t id;
};

__device__ __forceinline__ QueryIn load_query(const OrderArgs& A, int64_t i) {
    QueryIn q;
    const float* r = A.rays + i * 6;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        q.o[a] = r[a];
        q.d[a] = r[3 + a];
    }
    q.tm = A.tmax[i];
    q.id = A.ids[i];
    return q;
}

__device__ __forceinline__ uint32_t order_key(const OrderArgs& A, const QueryIn& q, uint32_t* fine) {
    *fine = fine_order_key(q.o, q.d, q.tm, q.id, A.objs, A.num_objects, A.fine_bits);
    return bucket_of_fine(*fine, A.fine_bits, A.bits, A.num_buckets);
}

// Pass 1: bucket of every query of the block's tile, counted in LDS; the
// counts of every bucket go to row `tile` of the table (tile-major).
constexpr int kOrderThreads = 1024;
constexpr int64_t kOrderTile = 8192;  // queries per block
__global__ __launch_bounds__(kOrderThreads) void order_count_kernel(OrderArgs A) {
    extern __shared__ uint32_t cnt[];
    if (A.zero_words && blockIdx.x == 0)
        for (int k = threadIdx.x; k < kTileCtrWords; k += blockDim.x) A.zero_words[k] = 0u;
    for (uint32_t k = threadIdx.x; k < A.num_buckets; k += blockDim.x) cnt[k] = 0;
    __syncthreads();
    const int64_t begin = (int64_t)blockIdx.x * A.tile, end = begin + A.tile < A.n ? begin + A.tile : A.n;
    for (int64_t i = begin + threadIdx.x; i < end; i += blockDim.x) {
        if (A.key_in) {  // keys given (found with the pairs): the bucket is a prefix of the key
            const uint32_t b = bucket_of_fine(A.key_in[i], A.fine_bits, A.bits, A.num_buckets);
            A.key[i] = (uint16_t)b;
            atomicAdd(&cnt[b], 1u);
            continue;
        }
        uint32_t fine;
        const QueryIn q = load_query(A, i);
        if (A.qrec) {  // the query as one 32-byte record, for the gathers through the order
            A.qrec[2 * i] = make_float4(q.o[0], q.o[1], q.o[2], q.d[0]);
            A.qrec[2 * i + 1] = make_float4(q.d[1], q.d[2], q.tm, __int_as_float(q.id));
        }
        const uint32_t b = order_key(A, q, &fine);
        A.key[i] = (uint16_t)b;
        if (!A.no_refine) A.fine[i] = fine;
        atomicAdd(&cnt[b], 1u);
    }
    __syncthreads();
    uint32_t* row = A.table + (int64_t)blockIdx.x * A.num_buckets;  // this tile's counts, every bucket
    for (uint32_t k = threadIdx.x; k < A.num_buckets; k += blockDim.x) row[k] = cnt[k];
}

// Pass 2: for every bucket, exclusive scan of its counts over the tiles (in
// place) and the bucket's total.  A block takes 16 buckets; its 16 x 64
// threads each own a segment of the tiles of one bucket: segment sums, their
// exclusive scan in LDS, then the segment's offsets.
constexpr int kScanBuckets = 16, kScanSegs = 64;
__global__ __launch_bounds__(kScanBuckets* kScanSegs) void order_tile_scan_kernel(uint32_t* table, int64_t tiles,
                                                                                  uint32_t nb, uint32_t* totals) {
    __shared__ uint32_t seg_sum[kScanSegs][kScanBuckets];
    const int lb = threadIdx.x % kScanBuckets, sg = threadIdx.x / kScanBuckets;
    const uint32_t b = blockIdx.x * kScanBuckets + lb;
    const int64_t per = (tiles + kScanSegs - 1) / kScanSegs;
    const int64_t t0 = sg * per, t1 = t0 + per < tiles ? t0 + per : tiles;
    uint32_t sum = 0;
    if (b < nb)
        for (int64_t t = t0; t < t1; ++t) sum += table[t * nb + b];
    seg_sum[sg][lb] = sum;
    __syncthreads();
    uint32_t run = 0;
    for (int j = 0; j < sg; ++j) run += seg_sum[j][lb];
    if (b < nb) {
        for (int64_t t = t0; t < t1; ++t) {
            const uint32_t v = table[t * nb + b];
            table[t * nb + b] = run;
            run += v;
        }
        if (sg == kScanSegs - 1) totals[b] = run;
    }
}

// Pass 3: every block turns the bucket totals into bucket offsets (an
// exclusive scan of at most 4097 values, redone by each block rather than in a
// one-block pass of its own), adds its tile's offsets, then ranks its queries
// inside (bucket, tile) with LDS counters and scatters to bucket offset + tile
// offset + rank.
constexpr int kMaxBuckets = 4097;
constexpr int kRankPer = (kMaxBuckets + kOrderThreads - 1) / kOrderThreads;  // buckets per thread
__global__ __launch_bounds__(kOrderThreads) void order_rank_kernel(OrderArgs A) {
    extern __shared__ uint32_t lds[];
    __shared__ uint32_t wave_sum[kOrderThreads / 64];
    const uint32_t nb = A.num_buckets;
    uint32_t* base = lds;     // nb offsets
    uint32_t* cur = lds + nb;  // nb rank counters
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t begin = (int64_t)blockIdx.x * A.tile, end = begin + A.tile < A.n ? begin + A.tile : A.n;
    constexpr int kPer = kOrderTile / kOrderThreads;
    uint32_t key[kPer], trow[kRankPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int64_t i = begin + tid + (int64_t)j * kOrderThreads;
        key[j] = i < end ? A.key[i] : 0u;
    }
    const uint32_t* row = A.table + (int64_t)blockIdx.x * nb;
#pragma unroll
    for (int j = 0; j < kRankPer; ++j) {
        const uint32_t k = tid + j * kOrderThreads;
        trow[j] = k < nb ? row[k] : 0u;
        if (k < nb) base[k] = A.block_sums[k];
    }
    __syncthreads();
    // Thread t owns buckets [t * kRankPer, (t + 1) * kRankPer).
    uint32_t v[kRankPer], sum = 0;
#pragma unroll
    for (int j = 0; j < kRankPer; ++j) {
        const uint32_t k = tid * kRankPer + j;
        v[j] = k < nb ? base[k] : 0u;
        sum += v[j];
    }
    uint32_t x = sum;  // inclusive scan over the wave
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) wave_sum[w] = x;
    __syncthreads();
    uint32_t run = x - sum;
    for (int j = 0; j < w; ++j) run += wave_sum[j];
#pragma unroll
    for (int j = 0; j < kRankPer; ++j) {
        const uint32_t k = tid * kRankPer + j;
        if (k < nb) base[k] = run;
        run += v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kRankPer; ++j) {
        const uint32_t k = tid + j * kOrderThreads;
        if (k < nb) {
            base[k] += trow[j];
            cur[k] = 0;
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int64_t i = begin + tid + (int64_t)j * kOrderThreads;
        if (i >= end) continue;
        const uint32_t b = key[j];
        const uint32_t r = atomicAdd(&cur[b], 1u);
        A.coarse[base[b] + r] = (uint32_t)i;
    }
}

// Pass 4: sort each window of kRefine consecutive entries of the bucket order
// by the finer key (object, 8 Morton bits per axis).  The window holds one or a
// few bucket runs, so its keys span a small range: keys are taken relative to
// the window's minimum and radix-sorted (a stable LDS radix sort, below) over
// only the bits that range needs.
constexpr int kRefineThreads = 256;
constexpr int kRefineItems = 16;
constexpr int kRefine = kRefineThreads * kRefineItems;
constexpr int kDigit = 4;  // radix bits per pass
constexpr int kBuckets = 1 << kDigit;

// Stable LSD radix sort of the block's kRefine (key, value) pairs on the key's
// low `bits` bits, in LDS.  Items are held blocked (thread t holds items
// 16 t .. 16 t + 15 of the current order).  One pass per 4-bit digit: every
// thread counts its items' digits in registers (16 counters of 8 bits packed
// in two 64-bit words) and writes them to column t of a [digit][thread]
// table; an exclusive scan of the table in digit-major order gives each
// (digit, thread) its first destination, and items go there in their order
// (the table entry plus the thread's running count of that digit), so that
// equal digits keep their relative order.  LDS indices are padded by one word
// per 32 (lds_pad) so that the strided accesses of the blocked arrangement
// fall into distinct banks.
__device__ __forceinline__ int lds_pad(int i) { return i + (i >> 5); }

struct RefineSortStorage {
    uint32_t key[kRefine + kRefine / 32];
    uint32_t val[kRefine + kRefine / 32];
    uint32_t table[kBuckets * kRefineThreads + kBuckets * kRefineThreads / 32];
    uint32_t part[kRefineThreads];
};

__device__ __forceinline__ uint32_t packed_count(uint64_t lo, uint64_t hi, uint32_t d) {
    return (uint32_t)(((d < 8 ? lo : hi) >> (8 * (d & 7))) & 0xffu);
}

__device__ __forceinline__ void refine_radix_sort(uint32_t (&key)[kRefineItems], uint32_t (&val)[kRefineItems],
                                                  RefineSortStorage& S, int bits) {
    static_assert(kBuckets == 16 && kRefineItems < 256, "8-bit packed counters of 16 digits");
    const int t = threadIdx.x;
    for (int shift = 0; shift < bits; shift += kDigit) {
        uint64_t lo = 0, hi = 0;
#pragma unroll
        for (int j = 0; j < kRefineItems; ++j) {
            const uint32_t d = (key[j] >> shift) & (kBuckets - 1);
            const uint64_t one = 1ull << (8 * (d & 7));
            lo += d < 8 ? one : 0ull;
            hi += d < 8 ? 0ull : one;
        }
#pragma unroll
        for (int b = 0; b < kBuckets; ++b) S.table[lds_pad(b * kRefineThreads + t)] = packed_count(lo, hi, b);
        __syncthreads();
        // exclusive scan of the table (kBuckets x kRefineThreads entries, digit-major):
        // thread t scans entries 16 t .. 16 t + 15, then the block scans the thread sums
        constexpr int per = kBuckets * kRefineThreads / kRefineThreads;
        uint32_t loc[per];
        uint32_t run = 0;
#pragma unroll
        for (int e = 0; e < per; ++e) {
            loc[e] = run;
            run += S.table[lds_pad(t * per + e)];
        }
        S.part[t] = run;
        __syncthreads();
        for (int off = 1; off < kRefineThreads; off <<= 1) {
            const uint32_t y = t >= off ? S.part[t - off] : 0u;
            __syncthreads();
            S.part[t] += y;
            __syncthreads();
        }
        const uint32_t base = t ? S.part[t - 1] : 0u;
#pragma unroll
        for (int e = 0; e < per; ++e) S.table[lds_pad(t * per + e)] = base + loc[e];
        __syncthreads();
        // scatter in order: the (digit, thread) start plus the thread's earlier items of that digit
        uint64_t rlo = 0, rhi = 0;
#pragma unroll
        for (int j = 0; j < kRefineItems; ++j) {
            const uint32_t d = (key[j] >> shift) & (kBuckets - 1);
            const uint32_t dst = S.table[lds_pad(d * kRefineThreads + t)] + packed_count(rlo, rhi, d);
            const uint64_t one = 1ull << (8 * (d & 7));
            rlo += d < 8 ? one : 0ull;
            rhi += d < 8 ? 0ull : one;
            S.key[lds_pad(dst)] = key[j];
            S.val[lds_pad(dst)] = val[j];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kRefineItems; ++j) {
            key[j] = S.key[lds_pad(t * kRefineItems + j)];
            val[j] = S.val[lds_pad(t * kRefineItems + j)];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kRefineThreads) void order_refine_kernel(OrderArgs A) {
    __shared__ RefineSortStorage storage;
    __shared__ uint32_t red_min[kRefineThreads / 64], red_max[kRefineThreads / 64];
    const int64_t w0 = (int64_t)blockIdx.x * kRefine;
    const int cnt = (int)(A.n - w0 < kRefine ? A.n - w0 : kRefine);
    uint32_t key[kRefineItems], val[kRefineItems];
    uint32_t mn = 0xffffffffu, mx = 0u;
#pragma unroll
    for (int j = 0; j < kRefineItems; ++j) {
        const int i = threadIdx.x * kRefineItems + j;  // blocked arrangement
        key[j] = 0xffffffffu;
        val[j] = 0xffffffffu;
        if (i < cnt) {
            val[j] = A.coarse[w0 + i];
            key[j] = A.fine[val[j]];
            mn = key[j] < mn ? key[j] : mn;
            mx = key[j] > mx ? key[j] : mx;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t a = __shfl_xor(mn, off), b = __shfl_xor(mx, off);
        mn = a < mn ? a : mn;
        mx = b > mx ? b : mx;
    }
    if ((threadIdx.x & 63) == 0) {
        red_min[threadIdx.x >> 6] = mn;
        red_max[threadIdx.x >> 6] = mx;
    }
    __syncthreads();
    mn = red_min[0];
    mx = red_max[0];
#pragma unroll
    for (int wv = 1; wv < kRefineThreads / 64; ++wv) {
        mn = red_min[wv] < mn ? red_min[wv] : mn;
        mx = red_max[wv] > mx ? red_max[wv] : mx;
    }
    const uint32_t range = mx - mn;  // valid keys map to [0, range]; padding stays 0xffffffff
    const int bits = range == 0u ? 0 : 32 - __builtin_clz(range);
    if (bits > 0) {
#pragma unroll
        for (int j = 0; j < kRefineItems; ++j)
            if (threadIdx.x * kRefineItems + j < cnt) key[j] -= mn;
        // padding keys (all ones) are >= every valid key in the low `bits` bits;
        // on a tie the stable sort keeps the padding, which comes last, last
        refine_radix_sort(key, val, storage, bits);
    }
#pragma unroll
    for (int j = 0; j < kRefineItems; ++j) {
        const int i = threadIdx.x * kRefineItems + j;
        if (i < cnt) A.perm[w0 + i] = val[j];
    }
}

int order_bits(int32_t num_objects) {
    int bits = 4;
    while (bits > 0 && ((int64_t)num_objects << (3 * bits)) > 4096) --bits;
    return bits;
}

// Fine key: object id and up to 8 Morton bits per axis in 31 bits, so that no
// hit's key equals the miss key 0xffffffff.
int order_fine_bits(int32_t num_objects) {
    int ob = 0;
    while (((int64_t)1 << ob) < num_objects) ++ob;
    int fb = (31 - ob) / 3;
    fb = fb > 8 ? 8 : fb;
    const int b = order_bits(num_objects);  // the bucket is a prefix of the fine key
    return fb < b ? b : fb;
}


struct OrderLayout {
    int64_t nb, tiles, table;
    size_t off_table, off_sums, off_key, off_fine, off_coarse, off_perm, total;
};

int order_bucket_bits(int32_t num_objects, int32_t max_bits) {
    const int b = order_bits(num_objects);
    return max_bits >= 0 && max_bits < b ? max_bits : b;
}

// Regions of the ordering workspace for `bits` bucket bits per axis; the
// workspace size is that of order_bits(num_objects), the largest.
static OrderLayout order_layout(int64_t n, int32_t num_objects, int bits) {
    OrderLayout L{};
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    L.nb = ((int64_t)num_objects << (3 * bits)) + 1;
    L.tiles = (n + kOrderTile - 1) / kOrderTile;
    L.table = L.nb * L.tiles;
    L.off_table = 0;
    L.off_sums = al(L.table * 4);  // bucket totals, then offsets
    L.off_key = L.off_sums + al(L.nb * 4);
    L.off_fine = L.off_key + al(n * 2);
    L.off_coarse = L.off_fine + al(n * 4);
    L.off_perm = L.off_coarse + al(n * 4);
    L.total = L.off_perm + al(n * 4);
    return L;
}

size_t order_workspace_bytes(int64_t n, int32_t num_objects) {
    if (num_objects > 4096) return 0;  // rejected by launch_order
    return order_layout(n, num_objects, order_bits(num_objects)).total;
}

hipError_t launch_order(OrderArgs A, void* ws, hipStream_t s, const uint32_t** perm_out) {
    if (A.num_objects > 4096) return hipErrorInvalidValue;
    A.bits = order_bucket_bits(A.num_objects, A.max_bits);
    const OrderLayout L = order_layout(A.n, A.num_objects, A.bits);
    A.fine_bits = order_fine_bits(A.num_objects);
    A.num_buckets = (uint32_t)L.nb;
    A.tile = kOrderTile;
    A.num_tiles = L.tiles;
    uint8_t* p = reinterpret_cast<uint8_t*>(ws);
    A.table = reinterpret_cast<uint32_t*>(p + L.off_table);
    A.block_sums = reinterpret_cast<uint32_t*>(p + L.off_sums);
    A.key = reinterpret_cast<uint16_t*>(p + L.off_key);
    A.fine = reinterpret_cast<uint32_t*>(p + L.off_fine);
    A.coarse = reinterpret_cast<uint32_t*>(p + L.off_coarse);
    if (A.key_in) A.fine = const_cast<uint32_t*>(A.key_in);  // the window sort reads the given keys
    if (!A.perm) A.perm = reinterpret_cast<uint32_t*>(p + L.off_perm);  // else the caller's buffer
    *perm_out = A.perm;
    const size_t lds = (size_t)L.nb * 4;
    hipLaunchKernelGGL(order_count_kernel, dim3((unsigned)L.tiles), dim3(kOrderThreads), lds, s, A);
    hipLaunchKernelGGL(order_tile_scan_kernel, dim3((unsigned)((L.nb + kScanBuckets - 1) / kScanBuckets)),
                       dim3(kScanBuckets * kScanSegs), 0, s, A.table, L.tiles, (uint32_t)L.nb, A.block_sums);
    if (A.no_refine) {
        A.coarse = A.perm;  // the bucket order is the result
        hipLaunchKernelGGL(order_rank_kernel, dim3((unsigned)L.tiles), dim3(kOrderThreads), 2 * lds, s, A);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(order_rank_kernel, dim3((unsigned)L.tiles), dim3(kOrderThreads), 2 * lds, s, A);
    hipLaunchKernelGGL(order_refine_kernel, dim3((unsigned)((A.n + kRefine - 1) / kRefine)), dim3(256), 0, s, A);
    return hipGetLastError();
}

}  // namespace nif
