// Top-level stage of a scene: (ray, object) pair expansion and per-ray
// combination.
//
// The method keeps the top-level traversal over the objects' boxes and issues
// one neural query per (ray, object) pair whose segment meets the object's
// AABB, in a separate pass before the network runs (Sec. 4.1); a ray is
// visible iff every such pair is visible, and a ray that meets no AABB is
// visible.  The hit rule is the query kernel's binary32 segment test
// (clip_segment), so a pair is emitted iff the query would not report a miss.
//
// Traversal.  The boxes form a two-level tree whose nodes are 64 wide, the
// width of a wavefront: level 1 holds up to 64 cluster boxes (or, with at most
// 64 objects, the object boxes themselves), level 2 the up-to-64 object boxes
// of each cluster, clusters being runs of 64 objects in the Morton order of
// their box centres.  A wave takes 64 consecutive rays.  Each lane clips its
// ray to the root box and bounds the clipped segment by a box with a relative
// margin; the union of the 64 lane boxes is the wave's bundle.  One node is
// then one compare per lane (lane j against child j) and a ballot, so the
// traversal is wave-uniform, with no per-ray stack and no divergence.  Every
// candidate object the ballots leave is tested by each lane against its own
// ray: a reciprocal-multiply slab test decides unless the box is grazed within
// 8 ulp, where the division test decides (see decide_hit).
//
// Why the bundle cull never drops a pair: if the binary32 test accepts box k,
// its interval [ta, tb] lies inside the root interval [T0, T1] computed with
// the widened reciprocal test (interval endpoints are monotone in the box
// bounds under rounding, and box k lies inside the root box), and the real
// point o + ta d lies within 2^-22 (|lo - o| + |hi - o|) of box k on every
// axis (two roundings in each slab quotient).  The lane box is the segment
// [T0, T1] with a margin of 2^-18 (|o| + |T0 d| + |T1 d| + |root bounds|) per
// axis, which covers both roundings and the rounding of the endpoints with
// room to spare, so box k overlaps the lane box and hence the bundle.
//
// Passes: (1) count: the hits of every ray (a 64-bit mask with at most 64
// objects, else a count) and the total of every block's contiguous run of
// 256-ray tiles; (2) an exclusive scan of the block totals in one block, which
// also writes the pair total; (3) emit, over the same runs: per tile a block
// scan of the ray counts, then the pairs in ray order, objects ascending
// within a ray.  The output is the same as a test of every box for every ray.
#include "nif_device.h"
#include "nif_order_key.h"
#include "nif_internal.h"

namespace nif {

constexpr int kPairTile = 256;  // rays per block tile: four waves of 64
constexpr int kPairScanThreads = 1024;
constexpr int kMaxPairBlocks = 8192;  // grid cap (1,024 compute units): sizes the per-object block table
constexpr float kUlp8 = 8.0f * 0x1p-24f;

struct RayPre {
    float o[3], d[3], inv[3], tm;
    bool fast;  // no direction component with 0 < |d| < 2^-100
};

// Boolean chains use & and | (not && and ||) so that they stay selects and
// do not become branches.
__device__ __forceinline__ RayPre ray_pre(const float o[3], const float d[3], float tm) {
    RayPre r;
    r.fast = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        r.o[a] = o[a];
        r.d[a] = d[a];
        r.inv[a] = __builtin_amdgcn_rcpf(d[a]);
        r.fast = r.fast & ((d[a] == 0.0f) | (fabsf(d[a]) >= 0x1p-100f));
    }
    r.tm = tm;
    return r;
}

// A ray that can have pairs: finite origin and direction, a non-zero
// direction, t_max not NaN and not negative (the query's domain rule).
__device__ __forceinline__ bool ray_valid(const float o[3], const float d[3], float tm) {
    bool ok = (d[0] != 0.0f) | (d[1] != 0.0f) | (d[2] != 0.0f);
#pragma unroll
    for (int a = 0; a < 3; ++a) ok = ok & (fabsf(o[a]) <= 0x1.fffffep127f) & (fabsf(d[a]) <= 0x1.fffffep127f);
    return ok & (tm >= 0.0f);
}

// Slab interval of a box with reciprocal multiplies (each end within 2^-22 of
// the binary32 quotient), before widening or narrowing.  Returns false when
// the ray is parallel to an axis and outside the box on it (exactly the
// division test's rule).
// Branch-free: every axis is computed and the parallel ones are selected
// away (their products may be NaN and are never used).
__device__ __forceinline__ bool slab_fast(const RayPre& r, const float lo[3], const float hi[3], float l[3],
                                          float h[3], bool con[3]) {
#pragma clang fp contract(off)
    bool inside = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        con[a] = r.d[a] != 0.0f;
        const float t0 = (lo[a] - r.o[a]) * r.inv[a];
        const float t1 = (hi[a] - r.o[a]) * r.inv[a];
        const bool lt = t0 < t1;
        l[a] = con[a] ? (lt ? t0 : t1) : -INFINITY;
        h[a] = con[a] ? (lt ? t1 : t0) : INFINITY;
        inside = inside & (con[a] | !((r.o[a] < lo[a]) | (r.o[a] > hi[a])));
    }
    return inside;
}

// Widened interval [ta, tb]: contains the division test's interval (the
// 2^-21 relative widening covers the 2^-22 error of the reciprocal form); an
// infinite end becomes NaN under widening and drops out of fmaxf / fminf,
// which can only widen further.
__device__ __forceinline__ void widened(const RayPre& r, const float l[3], const float h[3], const bool con[3],
                                        float& ta, float& tb) {
#pragma clang fp contract(off)
    (void)con;  // a parallel axis has l = -inf, h = +inf, which widen to themselves
    float tn = -INFINITY, tf = INFINITY;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        tn = fmaxf(tn, l[a] - kUlp8 * fabsf(l[a]));
        tf = fminf(tf, h[a] + kUlp8 * fabsf(h[a]));
    }
    ta = fmaxf(tn, 0.0f);
    tb = fminf(tf, r.tm);
}

// The binary32 division test's answer for one box, mostly without dividing:
// empty widened interval -> miss; non-empty narrowed interval (ends moved
// inwards by 2^-21, so contained in the division test's) -> hit; otherwise
// (a graze within 8 ulp, a non-finite or tiny slab end, a tiny direction
// component) the division test itself.  The reciprocal form runs in every
// lane without branches; lanes without r.fast take the division test.
__device__ __forceinline__ bool decide_hit(const RayPre& r, const float lo[3], const float hi[3]) {
#pragma clang fp contract(off)
    float l[3], h[3];
    bool con[3];
    const bool inside = slab_fast(r, lo, hi, l, h, con);
    float ta, tb;
    widened(r, l, h, con, ta, tb);
    const bool miss = !inside | !(ta <= tb);
    float tn = -INFINITY, tf = INFINITY;
    bool sure = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float al = fabsf(l[a]), ah = fabsf(h[a]);
        const bool ok = (al <= 0x1p100f) & (ah <= 0x1p100f) & ((al == 0.0f) | (al >= 0x1p-100f)) &
                        ((ah == 0.0f) | (ah >= 0x1p-100f));
        sure = sure & (!con[a] | ok);
        tn = con[a] ? fmaxf(tn, l[a] + kUlp8 * al) : tn;
        tf = con[a] ? fminf(tf, h[a] - kUlp8 * ah) : tf;
    }
    const bool hit = sure & (fmaxf(tn, 0.0f) <= fminf(tf, r.tm));
    bool res = !miss;
    if (!(r.fast & (miss | hit))) {
        float ta2, tb2;
        res = clip_segment(r.o, r.d, r.tm, lo, hi, ta2, tb2);
    }
    return res;
}

// Wave-wide reductions by DPP steps (quad permutes, row mirrors, row
// broadcasts): lane 63 ends with the result over all 64 lanes.  Floats are
// reduced as integers whose order is theirs (non-negative: the bit pattern;
// negative: its low 31 bits flipped), so each step is one integer min or max
// with no NaN quieting; a NaN input drops out, as it does from fminf / fmaxf.
// x from the DPP source lane; `id` (the operation's identity) in lanes of
// masked-out rows.
template <int CTRL, int ROWS>
__device__ __forceinline__ int32_t dpp_i(int32_t x, int32_t id) {
    return __builtin_amdgcn_update_dpp(id, x, CTRL, ROWS, 0xf, false);
}
__device__ __forceinline__ int32_t order_int(float v) {
    const int32_t i = __builtin_bit_cast(int32_t, v);
    return i >= 0 ? i : i ^ 0x7fffffff;
}
__device__ __forceinline__ float order_float(int32_t i) {
    return __builtin_bit_cast(float, i >= 0 ? i : i ^ 0x7fffffff);
}
template <typename Op>
__device__ __forceinline__ int32_t wave_reduce(int32_t x, int32_t id, Op op) {
    x = op(x, dpp_i<0xB1, 0xf>(x, id));
    x = op(x, dpp_i<0x4E, 0xf>(x, id));
    x = op(x, dpp_i<0x141, 0xf>(x, id));
    x = op(x, dpp_i<0x140, 0xf>(x, id));
    x = op(x, dpp_i<0x142, 0xa>(x, id));
    x = op(x, dpp_i<0x143, 0xc>(x, id));
    return __builtin_amdgcn_readlane(x, 63);
}
__device__ __forceinline__ float wave_min(float v) {
    const int32_t x = order_int(v != v ? INFINITY : v);
    return order_float(wave_reduce(x, INT32_MAX, [](int32_t a, int32_t b) { return a < b ? a : b; }));
}
__device__ __forceinline__ float wave_max(float v) {
    const int32_t x = order_int(v != v ? -INFINITY : v);
    return order_float(wave_reduce(x, INT32_MIN, [](int32_t a, int32_t b) { return a > b ? a : b; }));
}
// OR of a 64-bit value over the wave (in every lane: uniform).
__device__ __forceinline__ uint64_t wave_or64(uint64_t v) {
    auto op = [](int32_t a, int32_t b) { return a | b; };
    const uint32_t lo = (uint32_t)wave_reduce((int32_t)(uint32_t)v, 0, op);
    const uint32_t hi = (uint32_t)wave_reduce((int32_t)(uint32_t)(v >> 32), 0, op);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ float lane_f(float v, int j) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), j));
}
__device__ __forceinline__ float uniform_f(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

// One lane's ray: validity, the reciprocal form and its bundle box.
struct LaneRay {
    RayPre pre;
    bool active;
    float blo[3], bhi[3];  // conservative box of the root-clipped segment (empty: +inf / -inf)
};

// A lane's ray as read from memory (r >= n: a placeholder that is invalid).
struct RayIn {
    float o[3], d[3], tm;
};

__device__ __forceinline__ RayIn load_ray(const float* __restrict__ rays, const float* __restrict__ tmax, int64_t r,
                                          int64_t n) {
    RayIn q{{0, 0, 0}, {1, 0, 0}, -1.0f};
    if (r < n) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            q.o[a] = rays[r * 6 + a];
            q.d[a] = rays[r * 6 + 3 + a];
        }
        q.tm = tmax[r];
    }
    return q;
}

__device__ __forceinline__ LaneRay lane_ray(const RayIn& q, int64_t r, int64_t n, const PairTree& T) {
#pragma clang fp contract(off)
    LaneRay L;
    const float* o = q.o;
    const float* d = q.d;
    const float tm = q.tm;
    L.pre = ray_pre(o, d, tm);
    const bool valid = (r < n) & ray_valid(o, d, tm);  // invalid rays have no pairs
    // The root box clip, without branches.  A lane with a tiny direction
    // component is not culled (its bundle box is the whole root box); a
    // lane whose ray misses the root box meets no object box.
    float l[3], h[3];
    bool con[3];
    const bool inside = slab_fast(L.pre, T.root, T.root + 3, l, h, con);
    float t0, t1;
    widened(L.pre, l, h, con, t0, t1);
    L.active = valid & (!L.pre.fast | (inside & (t0 <= t1)));
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float p0 = o[a] + t0 * d[a], p1 = o[a] + t1 * d[a];
        float m = fabsf(o[a]) + fabsf(t0 * d[a]);
        m = m + fabsf(t1 * d[a]);
        m = m + fabsf(T.root[a]);
        m = m + fabsf(T.root[3 + a]);
        m = m * 0x1p-18f + 0x1p-100f;
        const float lo_c = fminf(p0, p1) - m, hi_c = fmaxf(p0, p1) + m;
        L.blo[a] = !L.active ? INFINITY : (L.pre.fast ? lo_c : T.root[a]);
        L.bhi[a] = !L.active ? -INFINITY : (L.pre.fast ? hi_c : T.root[3 + a]);
    }
    return L;
}

__device__ __forceinline__ bool overlaps(const float lo[3], const float hi[3], const float blo[3], const float bhi[3]) {
    return (lo[0] <= bhi[0]) & (lo[1] <= bhi[1]) & (lo[2] <= bhi[2]) & (hi[0] >= blo[0]) & (hi[1] >= blo[1]) &
           (hi[2] >= blo[2]);
}

// Level-1 entry of lane j: object j (one cluster) or cluster j.  Empty slots
// hold an empty box and id -1.
struct LaneBox {
    float lo[3], hi[3];
    int32_t id;
};

__device__ __forceinline__ LaneBox level1_box(const PairTree& T, int lane) {
    LaneBox b;
    const float* src = T.C == 1 ? T.mbox : T.cbox;
    const int cnt = T.C == 1 ? 64 : T.C;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        b.lo[a] = lane < cnt ? src[lane * 6 + a] : INFINITY;
        b.hi[a] = lane < cnt ? src[lane * 6 + 3 + a] : -INFINITY;
    }
    b.id = T.C == 1 ? (lane < 64 ? T.mid[lane] : -1) : (lane < T.C ? lane : -1);
    return b;
}

// Calls on_hit(i, object, lo, hi) for each of a lane's NR rays R[i] that the
// division test says meets that object's box; wave-uniform control flow.  The
// wave's bundle is the union of all its lanes' rays' boxes.  ONE: the tree
// has one level (at most 64 objects, T.C == 1).
template <bool ONE, int NR, typename F>
__device__ __forceinline__ void for_each_hit(const LaneRay* R, const LaneBox& B1, const PairTree& T, int lane,
                                             F&& on_hit) {
    float ulo[3], uhi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float lo = R[0].blo[a], hi = R[0].bhi[a];
#pragma unroll
        for (int i = 1; i < NR; ++i) {
            lo = fminf(lo, R[i].blo[a]);
            hi = fmaxf(hi, R[i].bhi[a]);
        }
        ulo[a] = uniform_f(wave_min(lo));
        uhi[a] = uniform_f(wave_max(hi));
    }
    if (!(ulo[0] <= uhi[0])) return;  // no active lane (wave-uniform)
    uint64_t cand = __ballot((B1.id >= 0) & overlaps(B1.lo, B1.hi, ulo, uhi));
    while (cand) {
        const int j = __builtin_ctzll(cand);
        cand &= cand - 1;
        if constexpr (ONE) {
            float lo[3], hi[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                lo[a] = lane_f(B1.lo[a], j);
                hi[a] = lane_f(B1.hi[a], j);
            }
            const int32_t k = __builtin_amdgcn_readlane(B1.id, j);
#pragma unroll
            for (int i = 0; i < NR; ++i)
                if (R[i].active && decide_hit(R[i].pre, lo, hi)) on_hit(i, k, lo, hi);
            continue;
        }
        // cluster j: its members, lane i holding member i
        LaneBox m;
        const int slot = j * 64 + lane;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            m.lo[a] = T.mbox[slot * 6 + a];
            m.hi[a] = T.mbox[slot * 6 + 3 + a];
        }
        m.id = T.mid[slot];
        uint64_t mc = __ballot((m.id >= 0) & overlaps(m.lo, m.hi, ulo, uhi));
        while (mc) {
            const int i = __builtin_ctzll(mc);
            mc &= mc - 1;
            float lo[3], hi[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                lo[a] = lane_f(m.lo[a], i);
                hi[a] = lane_f(m.hi[a], i);
            }
            const int32_t k = __builtin_amdgcn_readlane(m.id, i);
#pragma unroll
            for (int q = 0; q < NR; ++q)
                if (R[q].active && decide_hit(R[q].pre, lo, hi)) on_hit(q, k, lo, hi);
        }
    }
}

__device__ __forceinline__ uint32_t block_sum(uint32_t v, uint32_t* sh) {
    v = (uint32_t)wave_reduce((int32_t)v, 0, [](int32_t a, int32_t b) { return (int32_t)((uint32_t)a + (uint32_t)b); });
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[wave] = v;
    __syncthreads();
    const uint32_t t = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    return t;
}

// Exclusive scan over the block's 256 threads; the block total in `total`.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* sh, uint32_t& total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) sh[wave] = x;
    __syncthreads();
    uint32_t base = 0;
    for (int w = 0; w < wave; ++w) base += sh[w];
    total = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    return base + x - v;
}

// The count and emit passes run with the same grid; block b takes the
// contiguous tiles [tile_begin(tiles), tile_begin(tiles, 1)), so one total per
// block is all the scan between them needs.
__device__ __forceinline__ int64_t tile_begin(int64_t tiles, int next = 0) {
    return (int64_t)(blockIdx.x + next) * tiles / gridDim.x;
}

// Rounds of the early-out form (Sec. 7: once one object is found to occlude a
// ray, its remaining objects need not be queried): round 0 = every pair;
// round 1 = each ray's first pair only, the box it enters first (smallest
// t_a, then the smaller object id); round 2 = the pairs round 1 left out, of
// the rays still visible after it.  Rounds 1 and 2 together are round 0's
// pairs less those of rays occluded in round 1.
//
// Pass 1.  masks (K <= 64): bit k set iff the ray's pair with object k is
// emitted in this round; else counts (and, for rounds 1 and 2, the first
// object per ray in first_obj).
// ONE: one-level tree (T.C == 1); ROUNDS: round != 0.
template <bool ONE, bool ROUNDS>
__global__ __launch_bounds__(kPairTile) void pairs_count_kernel(const float* __restrict__ rays,
                                                                const float* __restrict__ tmax, int64_t n, PairTree T,
                                                                int32_t round, const uint8_t* __restrict__ ray_visible,
                                                                uint64_t* __restrict__ masks,
                                                                uint32_t* __restrict__ counts,
                                                                int32_t* __restrict__ first_obj,
                                                                uint32_t* __restrict__ block_sums,
                                                                uint32_t* __restrict__ obj_counts) {
    __shared__ uint32_t sh[4];
    __shared__ uint32_t hist[64];  // pairs of each object in the block (obj_counts)
    const int lane = threadIdx.x & 63;
    const LaneBox B1 = level1_box(T, lane);
    const int64_t tiles = (n + kPairTile - 1) / kPairTile;
    const int64_t t_end = tile_begin(tiles, 1);
    uint32_t block_total = 0;
    if (threadIdx.x < 64) hist[threadIdx.x] = 0;
    __syncthreads();
    if constexpr (!ROUNDS) {
        // Two rays per lane: a step covers two tiles (512 rays), wave w the 128
        // consecutive rays from 128 w, lane l rays l and 64 + l of them, so that
        // the bundle reductions and box reads serve 128 rays.  Rays past the
        // block's tiles (an odd last tile) are inactive.
        const int64_t rlim = t_end * kPairTile < n ? t_end * kPairTile : n;
        const int64_t wbase = (int64_t)(threadIdx.x >> 6) * 128 + lane;
        RayIn q_next[2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
            q_next[i] = load_ray(rays, tmax, tile_begin(tiles) * kPairTile + wbase + 64 * i, rlim);
        for (int64_t tile = tile_begin(tiles); tile < t_end; tile += 2) {
            LaneRay R[2];
            int64_t r[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                r[i] = tile * kPairTile + wbase + 64 * i;
                const RayIn q = q_next[i];  // the next step's rays are read before the work on these
                if (tile + 2 < t_end) q_next[i] = load_ray(rays, tmax, r[i] + 2 * kPairTile, rlim);
                R[i] = lane_ray(q, r[i], rlim, T);
            }
            uint64_t mk[2] = {0, 0};
            uint32_t c[2] = {0, 0};
            for_each_hit<ONE, 2>(R, B1, T, lane, [&](int i, int32_t k, const float*, const float*) {
                ++c[i];
                mk[i] |= 1ull << (k & 63);
            });
#pragma unroll
            for (int i = 0; i < 2; ++i)
                if (r[i] < rlim) {
                    if (masks) masks[r[i]] = mk[i];
                    else counts[r[i]] = c[i];
                }
            if (obj_counts) {  // per object: the wave's rays that meet it (ballots over the objects present)
                uint64_t present = wave_or64(mk[0] | mk[1]);
                while (present) {
                    const int k = __builtin_ctzll(present);
                    present &= present - 1;
                    const uint32_t cnt = (uint32_t)__popcll(__ballot((mk[0] >> k) & 1ull)) +
                                         (uint32_t)__popcll(__ballot((mk[1] >> k) & 1ull));
                    if (lane == 0) atomicAdd(&hist[k], cnt);
                }
            }
            block_total += block_sum(c[0] + c[1], sh);
        }
        if (threadIdx.x == 0) block_sums[blockIdx.x] = block_total;
        if (obj_counts) {  // object-major: entry k * gridDim.x + block
            __syncthreads();
            if (threadIdx.x < 64) obj_counts[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = hist[threadIdx.x];
        }
        return;
    }
    RayIn q_next = load_ray(rays, tmax, tile_begin(tiles) * kPairTile + threadIdx.x, n);
    for (int64_t tile = tile_begin(tiles); tile < t_end; ++tile) {
        const int64_t r = tile * kPairTile + threadIdx.x;
        const RayIn q = q_next;  // this tile's ray; the next tile's is read before the work on this one
        if (tile + 1 < t_end) q_next = load_ray(rays, tmax, r + kPairTile, n);
        const LaneRay R = lane_ray(q, r, n, T);
        uint64_t mk = 0;
        uint32_t c = 0;
        float best_ta = INFINITY;
        int32_t best_k = 0x7fffffff;
        for_each_hit<ONE, 1>(&R, B1, T, lane, [&](int, int32_t k, const float lo[3], const float hi[3]) {
            ++c;
            mk |= 1ull << (k & 63);
            if constexpr (ROUNDS) {  // the box entered first
                float ta, tb;
                (void)clip_segment(R.pre.o, R.pre.d, R.pre.tm, lo, hi, ta, tb);
                if (ta < best_ta || (ta == best_ta && k < best_k)) {
                    best_ta = ta;
                    best_k = k;
                }
            }
        });
        if (ROUNDS && round == 1 && c) {
            c = 1;
            mk = 1ull << (best_k & 63);
        } else if (ROUNDS && round == 2 && c) {
            if (r < n && ray_visible[r]) {
                c -= 1;
                mk &= ~(1ull << (best_k & 63));
            } else {
                c = 0;
                mk = 0;
            }
        }
        if (r < n) {
            if (masks) masks[r] = mk;
            else counts[r] = c;
            if (first_obj) first_obj[r] = best_k;
        }
        block_total += block_sum(c, sh);
    }
    if (threadIdx.x == 0) block_sums[blockIdx.x] = block_total;
}

// Pass 2: exclusive scan of the per-block totals (at most a few thousand
// values, one block: each thread sums a short contiguous run, a scan of the
// run totals, then the runs are written out); the pair total.
__global__ __launch_bounds__(kPairScanThreads) void pairs_block_scan_kernel(const uint32_t* __restrict__ sums,
                                                                            int64_t nb,
                                                                            uint64_t* __restrict__ offs,
                                                                            int64_t* __restrict__ total) {
    __shared__ uint64_t part[kPairScanThreads];
    const int t = threadIdx.x;
    const int64_t per = (nb + kPairScanThreads - 1) / kPairScanThreads;
    const int64_t b = t * per, e = b + per < nb ? b + per : nb;
    uint64_t s = 0;
    for (int64_t i = b; i < e; ++i) s += sums[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < kPairScanThreads; off <<= 1) {  // inclusive scan of the run totals
        const uint64_t y = t >= off ? part[t - off] : 0ull;
        __syncthreads();
        part[t] += y;
        __syncthreads();
    }
    uint64_t run = t ? part[t - 1] : 0ull;
    for (int64_t i = b; i < e; ++i) {
        offs[i] = run;
        run += sums[i];
    }
    if (t == kPairScanThreads - 1) *total = (int64_t)part[t];
}

// Where the pairs go: separate arrays (pair_rays, pair_tmax, pair_ids), or
// 32-byte query records {o, d.x}, {d.y, d.z, t_max, object id bits} with,
// optionally, each pair's ordering key (the ordering's fine key, so that the
// ordering need not read the pairs again; with object_keys, for an ordering
// by object alone, the object's part of it with the Morton bits zero);
// pair_ray always.
struct PairOut {
    float* pair_rays;
    float* pair_tmax;
    int32_t* pair_ids;
    uint32_t* pair_ray;
    float4* rec;
    uint32_t* key;
    const ObjDev* objs;
    int32_t K;
    int32_t fine_bits;
    bool object_keys;
};

// The ordering key of a pair (a valid query that meets its box).
__device__ __forceinline__ uint32_t pair_key(const float o[3], const float d[3], float tm, int32_t k,
                                             const ObjDev* __restrict__ objs, const PairOut& out) {
    return out.object_keys ? (uint32_t)k << (3 * out.fine_bits) : fine_order_key(o, d, tm, k, objs, out.K, out.fine_bits);
}

__device__ __forceinline__ void write_pair(int64_t p, const float o[3], const float d[3], float tm, int32_t k,
                                           uint32_t ray, const PairOut& out) {
    if (out.rec) {
        out.rec[2 * p] = make_float4(o[0], o[1], o[2], d[0]);
        out.rec[2 * p + 1] = make_float4(d[1], d[2], tm, __int_as_float(k));
        if (out.key) out.key[p] = pair_key(o, d, tm, k, out.objs, out);
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            out.pair_rays[p * 6 + a] = o[a];
            out.pair_rays[p * 6 + 3 + a] = d[a];
        }
        out.pair_tmax[p] = tm;
        out.pair_ids[p] = k;
    }
    out.pair_ray[p] = ray;
}

__device__ __forceinline__ int32_t pair_id(const PairOut& out, int64_t p) {
    return out.rec ? __float_as_int(reinterpret_cast<const float*>(out.rec)[8 * p + 7]) : out.pair_ids[p];
}

__device__ __forceinline__ void set_pair_id(const PairOut& out, int64_t p, int32_t k) {
    if (out.rec)
        reinterpret_cast<float*>(out.rec)[8 * p + 7] = __int_as_float(k);
    else
        out.pair_ids[p] = k;
}

// Records of up to kPairStage pairs of a tile are staged in LDS and stored as
// one contiguous run (each lane's own pairs are scattered across the tile's
// output, 32 bytes apart per pair of a ray).
constexpr int kPairStage = 512;

// Pass 3 with masks (at most 64 objects): ascending set bits.  Masks are
// read two tiles ahead and rays (of rays with pairs) one tile ahead, so that
// a block's serial chain of tiles waits on memory as little as possible; the
// object boxes for the keys are read from LDS.
__global__ __launch_bounds__(kPairTile) void pairs_emit_mask_kernel(
    const float* __restrict__ rays, const float* __restrict__ tmax, int64_t n, const uint64_t* __restrict__ masks,
    const uint64_t* __restrict__ offs, int64_t max_pairs, PairOut out) {
    __shared__ uint32_t sh[4];
    __shared__ float4 srec[2 * kPairStage];
    __shared__ uint32_t sray[kPairStage];
    __shared__ ObjDev sobj[64];
    if (out.key && !out.object_keys)
        for (int i = threadIdx.x; i < out.K; i += kPairTile) sobj[i] = out.objs[i];
    __syncthreads();
    const int64_t tiles = (n + kPairTile - 1) / kPairTile;
    const int64_t t_end = tile_begin(tiles, 1);
    int64_t run = (int64_t)offs[blockIdx.x];
    int64_t tile = tile_begin(tiles);
    auto mask_at = [&](int64_t t) -> uint64_t {
        const int64_t r = t * kPairTile + threadIdx.x;
        return t < t_end && r < n ? masks[r] : 0ull;
    };
    auto ray_at = [&](int64_t t, uint64_t m) -> RayIn {  // read only for rays with pairs
        return load_ray(rays, tmax, m ? t * kPairTile + threadIdx.x : n, n);
    };
    // pipeline: masks two tiles ahead, rays one tile ahead
    uint64_t mk_next = mask_at(tile);
    RayIn q_next = ray_at(tile, mk_next);
    uint64_t mk_next2 = mask_at(tile + 1);
    for (; tile < t_end; ++tile) {
        const int64_t r = tile * kPairTile + threadIdx.x;
        uint64_t mk = mk_next;
        const RayIn q = q_next;
        mk_next = mk_next2;
        q_next = ray_at(tile + 1, mk_next);
        mk_next2 = mask_at(tile + 2);
        const uint32_t c = (uint32_t)__popcll(mk);
        const float* o = q.o;
        const float* d = q.d;
        const float tm = q.tm;
        uint32_t tile_total;
        const uint32_t lp = block_excl_scan(c, sh, tile_total);
        const int64_t base = run;
        run += tile_total;
        // block-uniform: stage the tile's records when they fit and none is cut off
        const bool stage = out.rec && tile_total <= (uint32_t)kPairStage && base + tile_total <= max_pairs;
        int64_t p = base + lp;
        if (c != 0 && p < max_pairs) {
            if (stage) {
                for (uint32_t j = lp; mk; ++j) {
                    const int k = __builtin_ctzll(mk);
                    mk &= mk - 1;
                    srec[2 * j] = make_float4(o[0], o[1], o[2], d[0]);
                    srec[2 * j + 1] = make_float4(d[1], d[2], tm, __int_as_float(k));
                    sray[j] = (uint32_t)r;
                }
            } else {
                PairOut o2 = out;
                o2.objs = sobj;
                while (mk && p < max_pairs) {
                    const int k = __builtin_ctzll(mk);
                    mk &= mk - 1;
                    write_pair(p++, o, d, tm, k, (uint32_t)r, o2);
                }
            }
        }
        if (stage) {  // stores of the tile's run; the keys with one lane per pair, not per ray
            __syncthreads();
            for (uint32_t i = threadIdx.x; i < 2 * tile_total; i += kPairTile) out.rec[2 * base + i] = srec[i];
            for (uint32_t i = threadIdx.x; i < tile_total; i += kPairTile) {
                out.pair_ray[base + i] = sray[i];
                if (out.key) {
                    const float4 a = srec[2 * i], b = srec[2 * i + 1];
                    const float qo[3] = {a.x, a.y, a.z}, qd[3] = {a.w, b.x, b.y};
                    out.key[base + i] = pair_key(qo, qd, b.z, __float_as_int(b.w), sobj, out);
                }
            }
            __syncthreads();
        }
    }
}

// Object bases: exclusive scan of the 64 object totals in 64 bits (wave 0 of
// a block, lane k for object k; the wave-wide total in every lane).
__device__ __forceinline__ uint64_t object_base(const uint32_t* __restrict__ obj_tot, int lane, uint64_t& all) {
    const uint64_t v = obj_tot[lane];
    uint64_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    all = __shfl(x, 63);
    return x - v;
}

// Pass 3 grouped by object (at most 64 objects): the pairs of object k go to
// base(k) + local[k * gridDim.x + block] onwards (base(k): the pairs of the
// objects before k; local: the scan of the per-object block counts), in ray
// order within the block, so that the whole output is grouped
// by object and in ray order within each object.  Per tile, each wave counts
// its lanes of each object present (ballots), the waves' counts give each
// lane its place, and the block's running count per object advances.
__global__ __launch_bounds__(kPairTile) void pairs_emit_grouped_kernel(
    const float* __restrict__ rays, const float* __restrict__ tmax, int64_t n, const uint64_t* __restrict__ masks,
    const uint32_t* __restrict__ local, const uint32_t* __restrict__ obj_tot, int32_t K, int64_t max_pairs,
    float4* __restrict__ rec, uint32_t* __restrict__ pair_ray, int64_t* __restrict__ total,
    int64_t* __restrict__ obj_off) {
    __shared__ uint64_t base[64];   // where the block's pairs of each object start
    __shared__ uint32_t run[64];    // the block's pairs of each object in earlier tiles
    __shared__ uint32_t wc[4][64];  // this tile's pairs of each object per wave
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x < 64) {  // wave 0: where each object's pairs start, and this block's part of them
        uint64_t all;
        const uint64_t ob = object_base(obj_tot, lane, all);
        base[lane] = ob + local[(int64_t)lane * gridDim.x + blockIdx.x];
        run[lane] = 0;
        if (blockIdx.x == 0) {  // K <= 64: lanes 0..K-1 the objects' first pairs, lane 0 also the total
            if (obj_off && lane < K) obj_off[lane] = (int64_t)ob;
            if (lane == 0) {
                *total = (int64_t)all;
                if (obj_off) obj_off[K] = (int64_t)all;
            }
        }
    }
    const uint64_t lt = (1ull << lane) - 1ull;  // lanes below this one
    const int64_t tiles = (n + kPairTile - 1) / kPairTile;
    const int64_t t_end = tile_begin(tiles, 1);
    int64_t tile = tile_begin(tiles);
    auto mask_at = [&](int64_t t) -> uint64_t {
        const int64_t r = t * kPairTile + threadIdx.x;
        return t < t_end && r < n ? masks[r] : 0ull;
    };
    auto ray_at = [&](int64_t t, uint64_t m) -> RayIn {  // read only for rays with pairs
        return load_ray(rays, tmax, m ? t * kPairTile + threadIdx.x : n, n);
    };
    uint64_t mk_next = mask_at(tile);
    RayIn q_next = ray_at(tile, mk_next);
    uint64_t mk_next2 = mask_at(tile + 1);
    for (; tile < t_end; ++tile) {
        const int64_t r = tile * kPairTile + threadIdx.x;
        const uint64_t mk = mk_next;
        const RayIn q = q_next;
        mk_next = mk_next2;
        q_next = ray_at(tile + 1, mk_next);
        mk_next2 = mask_at(tile + 2);
        wc[wave][lane] = 0;
        __syncthreads();
        const uint64_t present = wave_or64(mk);
        for (uint64_t pm = present; pm; pm &= pm - 1) {
            const int k = __builtin_ctzll(pm);
            const uint64_t b = __ballot((mk >> k) & 1ull);
            if (lane == 0) wc[wave][k] = (uint32_t)__popcll(b);
        }
        __syncthreads();
        for (uint64_t pm = present; pm; pm &= pm - 1) {
            const int k = __builtin_ctzll(pm);
            const uint64_t b = __ballot((mk >> k) & 1ull);
            if ((mk >> k) & 1ull) {
                uint64_t p = base[k] + run[k] + (uint64_t)__popcll(b & lt);
                for (int w = 0; w < wave; ++w) p += wc[w][k];
                if ((int64_t)p < max_pairs) {
                    rec[2 * p] = make_float4(q.o[0], q.o[1], q.o[2], q.d[0]);
                    rec[2 * p + 1] = make_float4(q.d[1], q.d[2], q.tm, __int_as_float(k));
                    pair_ray[p] = (uint32_t)r;
                }
            }
        }
        __syncthreads();
        if (threadIdx.x < 64) run[threadIdx.x] += wc[0][threadIdx.x] + wc[1][threadIdx.x] + wc[2][threadIdx.x] + wc[3][threadIdx.x];
        __syncthreads();
    }
}

// Scan of the per-object block counts, one block per object (64 blocks):
// offs[k * blocks + b] = the pairs of object k in blocks before b, in u32
// first; obj_tot[k] = object k's pairs.
constexpr int kObjScanThreads = 256;
__global__ __launch_bounds__(kObjScanThreads) void obj_scan_kernel(const uint32_t* __restrict__ counts,
                                                                   int32_t blocks, uint32_t* __restrict__ local,
                                                                   uint32_t* __restrict__ obj_tot) {
    __shared__ uint32_t part[kObjScanThreads];
    const int t = threadIdx.x, k = blockIdx.x;
    const int per = (blocks + kObjScanThreads - 1) / kObjScanThreads;
    const uint32_t* c = counts + (int64_t)k * blocks;
    uint32_t s = 0;
    for (int i = t * per; i < (t + 1) * per && i < blocks; ++i) s += c[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < kObjScanThreads; off <<= 1) {
        const uint32_t y = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += y;
        __syncthreads();
    }
    uint32_t run = t ? part[t - 1] : 0u;
    for (int i = t * per; i < (t + 1) * per && i < blocks; ++i) {
        local[(int64_t)k * blocks + i] = run;
        run += c[i];
    }
    if (t == kObjScanThreads - 1) obj_tot[k] = part[t];
}


// Pass 3 with more than 64 objects: the traversal again, pairs written in
// traversal order, then the ray's written ids sorted ascending in place (the
// other fields are the same for every pair of a ray).
__global__ __launch_bounds__(kPairTile) void pairs_emit_tree_kernel(
    const float* __restrict__ rays, const float* __restrict__ tmax, int64_t n, PairTree T, int32_t round,
    const int32_t* __restrict__ first_obj, const uint32_t* __restrict__ counts, const uint64_t* __restrict__ offs,
    int64_t max_pairs, PairOut out) {
    __shared__ uint32_t sh[4];
    const int lane = threadIdx.x & 63;
    const LaneBox B1 = level1_box(T, lane);
    const int64_t tiles = (n + kPairTile - 1) / kPairTile;
    int64_t run = (int64_t)offs[blockIdx.x];
    for (int64_t tile = tile_begin(tiles); tile < tile_begin(tiles, 1); ++tile) {
        const int64_t r = tile * kPairTile + threadIdx.x;
        const uint32_t c = r < n ? counts[r] : 0u;
        uint32_t tile_total;
        const int64_t p0 = run + block_excl_scan(c, sh, tile_total);
        run += tile_total;
        const LaneRay R = lane_ray(load_ray(rays, tmax, r, n), r, n, T);
        const int32_t first = round && r < n ? first_obj[r] : -1;
        int64_t p = p0;
        for_each_hit<false, 1>(&R, B1, T, lane, [&](int, int32_t k, const float*, const float*) {
            // round 1: the first object only; round 2: the others (a ray with c = 0 writes none)
            if ((round == 1 && k != first) || (round == 2 && k == first) || p >= p0 + (int64_t)c) return;
            if (p < max_pairs) write_pair(p, R.pre.o, R.pre.d, R.pre.tm, k, (uint32_t)r, out);
            ++p;
        });
        const int64_t e = p < max_pairs ? p : max_pairs;
        for (int64_t i = p0 + 1; i < e; ++i) {  // insertion sort of the ray's ids, keys along
            const int32_t v = pair_id(out, i);
            const uint32_t kv = out.key ? out.key[i] : 0u;
            int64_t j = i - 1;
            while (j >= p0 && pair_id(out, j) > v) {
                set_pair_id(out, j + 1, pair_id(out, j));
                if (out.key) out.key[j + 1] = out.key[j];
                --j;
            }
            set_pair_id(out, j + 1, v);
            if (out.key) out.key[j + 1] = kv;
        }
    }
}

__global__ void pairs_zero_total_kernel(int64_t* total) {
    if (threadIdx.x == 0) *total = 0;
}

// Ray visibility: 1 unless some pair of the ray has visibility < 0.5.  The
// initial ones go out as 16-byte stores from the first 16-byte boundary on;
// the bytes before it and after the last whole 16 bytes one by one.
__global__ void combine_init_kernel(uint8_t* ray_visible, int64_t n_rays) {
    const int64_t lead = (int64_t)((16u - (uint32_t)(reinterpret_cast<uintptr_t>(ray_visible) & 15u)) & 15u);
    const int64_t head = lead < n_rays ? lead : n_rays;
    const int64_t body = (n_rays - head) / 16;
    const int64_t tail0 = head + body * 16;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint4* v = reinterpret_cast<uint4*>(ray_visible + head);
    for (int64_t i = t; i < body; i += stride) v[i] = make_uint4(0x01010101u, 0x01010101u, 0x01010101u, 0x01010101u);
    const int64_t edge = head + (n_rays - tail0);
    for (int64_t i = t; i < edge; i += stride) ray_visible[i < head ? i : tail0 + (i - head)] = 1;
}

__global__ void combine_pairs_kernel(const uint32_t* __restrict__ pair_ray, const float* __restrict__ vis,
                                     int64_t n_pairs, int64_t n_rays, uint8_t* __restrict__ ray_visible) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n_pairs; p += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t r = pair_ray[p];
        if (vis[p] < 0.5f && r < n_rays) ray_visible[r] = 0;  // every writer stores the same value
    }
}

// The same with four pairs per thread and 16-byte loads (pair_ray and vis
// 16-byte aligned); the last n_pairs % 4 pairs one per thread.
__global__ void combine_pairs4_kernel(const uint4* __restrict__ pair_ray, const float4* __restrict__ vis,
                                      int64_t n_pairs, int64_t n_rays, uint8_t* __restrict__ ray_visible) {
    const int64_t n4 = n_pairs / 4;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
        const uint4 r = pair_ray[i];
        const float4 v = vis[i];
        if (v.x < 0.5f && r.x < n_rays) ray_visible[r.x] = 0;
        if (v.y < 0.5f && r.y < n_rays) ray_visible[r.y] = 0;
        if (v.z < 0.5f && r.z < n_rays) ray_visible[r.z] = 0;
        if (v.w < 0.5f && r.w < n_rays) ray_visible[r.w] = 0;
    }
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n_pairs - 4 * n4) {
        const int64_t p = 4 * n4 + t;
        const uint32_t r = reinterpret_cast<const uint32_t*>(pair_ray)[p];
        if (reinterpret_cast<const float*>(vis)[p] < 0.5f && r < n_rays) ray_visible[r] = 0;
    }
}

// Depth output of primary-ray queries (Sec. 7: the network can encode the
// first hit's depth): the visibility output read as the normalised position
// of the hit in the query's segment.
__global__ void depth_from_visibility_kernel(const float* __restrict__ rays, const int32_t* __restrict__ ids,
                                             const float* __restrict__ tmax, const float* __restrict__ vis, int64_t n,
                                             const ObjDev* __restrict__ objs, int32_t K, float* __restrict__ depth) {
#pragma clang fp contract(off)
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float o[3], d[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            o[a] = rays[i * 6 + a];
            d[a] = rays[i * 6 + 3 + a];
        }
        const float tm = tmax[i];
        const int32_t id = ids[i];
        float out = NAN;
        if (valid_query(o, d, tm, id, K)) {
            float ta, tb;
            out = clip_segment(o, d, tm, objs[id].lo, objs[id].hi, ta, tb) ? ta + vis[i] * (tb - ta) : INFINITY;
        }
        depth[i] = out;
    }
}

hipError_t launch_depth_from_visibility(const float* rays, const int32_t* ids, const float* tmax, const float* vis,
                                        int64_t n, const ObjDev* objs, int32_t K, float* depth, int num_cus,
                                        hipStream_t s) {
    int64_t b = (n + 255) / 256;
    if (b > (int64_t)num_cus * 16) b = (int64_t)num_cus * 16;
    hipLaunchKernelGGL(depth_from_visibility_kernel, dim3((unsigned)(b > 0 ? b : 1)), dim3(256), 0, s, rays, ids, tmax,
                       vis, n, objs, K, depth);
    return hipGetLastError();
}

static size_t al256(size_t b) { return (b + 255) / 256 * 256; }

// masks (8 B per ray) or counts (4 B), per-block totals (4 B) and offsets
// (8 B), first objects (4 B per ray, more than 64 objects only).  Sized by
// tiles, which bounds the block count.
// Masks (at most 64 objects) or counts, block totals and their offsets, then
// (masks only, for the grouped form) the per-object block counts, their scan
// within each object and the 64 object totals; or (more than 64 objects) the
// first objects.
size_t pairs_workspace_bytes(int64_t n_rays, int32_t K) {
    const int64_t tiles = (n_rays + kPairTile - 1) / kPairTile;
    const int64_t blocks = tiles < kMaxPairBlocks ? tiles : kMaxPairBlocks;
    return al256((size_t)n_rays * (K <= 64 ? 8 : 4)) + al256((size_t)tiles * 4) + al256((size_t)tiles * 8) +
           (K <= 64 ? 2 * al256((size_t)64 * blocks * 4) + 256 : al256((size_t)n_rays * 4));
}

static unsigned grid_for(int64_t n, int threads) {
    const int64_t b = (n + threads - 1) / threads;
    return (unsigned)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

hipError_t launch_expand_pairs(const float* rays, const float* tmax, int64_t n, const PairTree& T, int32_t K,
                               int num_cus, int32_t round, const uint8_t* ray_visible, int64_t max_pairs,
                               float* pair_rays, float* pair_tmax, int32_t* pair_ids, uint32_t* pair_ray,
                               int64_t* total, void* ws, hipStream_t s, float4* rec, uint32_t* keys,
                               const ObjDev* objs, bool object_keys, bool grouped, int64_t* obj_off) {
    if (n == 0) {
        hipLaunchKernelGGL(pairs_zero_total_kernel, dim3(1), dim3(64), 0, s, total);
        return hipGetLastError();
    }
    const int64_t tiles = (n + kPairTile - 1) / kPairTile;
    uint8_t* p = reinterpret_cast<uint8_t*>(ws);
    const bool use_mask = K <= 64;
    uint64_t* masks = use_mask ? reinterpret_cast<uint64_t*>(p) : nullptr;
    uint32_t* counts = use_mask ? nullptr : reinterpret_cast<uint32_t*>(p);
    p += al256((size_t)n * (use_mask ? 8 : 4));
    uint32_t* sums = reinterpret_cast<uint32_t*>(p);
    p += al256((size_t)tiles * 4);
    uint64_t* offs = reinterpret_cast<uint64_t*>(p);
    p += al256((size_t)tiles * 8);
    int32_t* first = use_mask ? nullptr : reinterpret_cast<int32_t*>(p);
    int64_t cap = (int64_t)num_cus * 8;  // persistent blocks
    cap = cap < kMaxPairBlocks ? cap : kMaxPairBlocks;
    const unsigned blocks = (unsigned)(tiles < cap ? tiles : cap);
    if (grouped && (!use_mask || round)) return hipErrorInvalidValue;  // checked by the caller
    // grouped: per-object block counts, their scan within each object, the
    // object totals and bases
    uint32_t* obj_counts = grouped ? reinterpret_cast<uint32_t*>(p) : nullptr;
    uint32_t* obj_local = grouped ? reinterpret_cast<uint32_t*>(p + al256((size_t)64 * blocks * 4)) : nullptr;
    uint32_t* obj_tot = grouped ? reinterpret_cast<uint32_t*>(p + 2 * al256((size_t)64 * blocks * 4)) : nullptr;
    auto count = T.C == 1 ? (round ? pairs_count_kernel<true, true> : pairs_count_kernel<true, false>)
                          : (round ? pairs_count_kernel<false, true> : pairs_count_kernel<false, false>);
    hipLaunchKernelGGL(count, dim3(blocks), dim3(kPairTile), 0, s, rays, tmax, n, T, round, ray_visible, masks, counts,
                       round ? first : nullptr, sums, obj_counts);
    if (grouped) {
        hipLaunchKernelGGL(obj_scan_kernel, dim3(64), dim3(kObjScanThreads), 0, s, obj_counts, (int32_t)blocks,
                           obj_local, obj_tot);
        hipLaunchKernelGGL(pairs_emit_grouped_kernel, dim3(blocks), dim3(kPairTile), 0, s, rays, tmax, n, masks,
                           obj_local, obj_tot, K, max_pairs, rec, pair_ray, total, obj_off);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(pairs_block_scan_kernel, dim3(1), dim3(kPairScanThreads), 0, s, sums, (int64_t)blocks, offs,
                       total);
    const PairOut out{pair_rays, pair_tmax, pair_ids, pair_ray, rec, keys, objs, K, order_fine_bits(K), object_keys};
    if (use_mask)
        hipLaunchKernelGGL(pairs_emit_mask_kernel, dim3(blocks), dim3(kPairTile), 0, s, rays, tmax, n, masks, offs,
                           max_pairs, out);
    else
        hipLaunchKernelGGL(pairs_emit_tree_kernel, dim3(blocks), dim3(kPairTile), 0, s, rays, tmax, n, T, round, first,
                           counts, offs, max_pairs, out);
    return hipGetLastError();
}

hipError_t launch_combine_pairs(const uint32_t* pair_ray, const float* vis, int64_t n_pairs, int64_t n_rays,
                                uint8_t* ray_visible, bool init, hipStream_t s) {
    if (init && n_rays > 0)
        hipLaunchKernelGGL(combine_init_kernel, dim3(grid_for((n_rays + 15) / 16, 256)), dim3(256), 0, s, ray_visible,
                           n_rays);
    if (n_pairs > 0) {
        if (((reinterpret_cast<uintptr_t>(pair_ray) | reinterpret_cast<uintptr_t>(vis)) & 15u) == 0)
            hipLaunchKernelGGL(combine_pairs4_kernel, dim3(grid_for((n_pairs + 3) / 4, 256)), dim3(256), 0, s,
                               reinterpret_cast<const uint4*>(pair_ray), reinterpret_cast<const float4*>(vis), n_pairs,
                               n_rays, ray_visible);
        else
            hipLaunchKernelGGL(combine_pairs_kernel, dim3(grid_for(n_pairs, 256)), dim3(256), 0, s, pair_ray, vis,
                               n_pairs, n_rays, ray_visible);
    }
    return hipGetLastError();
}

}  // namespace nif
