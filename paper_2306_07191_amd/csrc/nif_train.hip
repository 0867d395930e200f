// Online training step (Sec. 4.2 and Sec. 5 "Training" of the paper: latents
// and weights optimised jointly with Adam by back-propagation through the MLP
// and the grid interpolation, Sec. 3.1 / Fig. 2).
//
// Loss: binary cross-entropy on the logit, averaged over the B queries of the
// batch that meet their AABB and use the trained MLP:
//   L = (1/B) sum [softplus(z) - t z],   dL/dz = (sigmoid(z) - t) / B.
// Everything below accumulates the unscaled (sigmoid(z) - t); the 1/B factor
// is applied when the gradients are consumed (B is only known on the device).
// Upstream-gradient mode (grad_y set, no labels, no Adam): dL/dz = g_y
// sigmoid(z) (1 - sigmoid(z)) for a given dL/dy per query, and no 1/B factor.
//
// Kernels:
//  T1 train_fb_kernel: per wave 32 queries, two lanes per query (the query
//     kernel's mapping).  Clip + encode, forward on binary32 MFMA keeping every
//     layer input (activations) and, after the loss, every layer's output
//     delta in a [feature][slot] workspace; the deltas are propagated with the
//     transposed weight image; the feature gradient g_x comes out in the lane
//     that encoded those features, which then scatter-adds weight * g_x into
//     the grid gradient and flags the touched chunks: coarse levels through a
//     per-block LDS table flushed once per block, fine levels by binary32
//     atomics.
//  T2 train_dw_kernel: dW_j = sum over slots of delta_j x input_j (split-K on
//     binary32 MFMA, one 32x32 tile per wave, deterministic per-chunk partials),
//     then train_dw_reduce_kernel sums the partials in chunk order.
//  T3 adam_mlp_kernel: dense Adam on the MLP master (binary32).
//  T4 adam_grid_kernel: Adam on latents whose gradient is non-zero this step,
//     found through the dirty chunk flags; clears gradient and flags.
#include <hip/hip_fp16.h>

#include "nif_device.h"
#include "nif_internal.h"

namespace nif {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

#define GLOBAL __attribute__((address_space(1)))

__device__ __forceinline__ f32x4 load4(const float* p) { return *reinterpret_cast<const f32x4*>(p); }

__device__ __forceinline__ int cell_coord_t(float u, float fN, int N, float& w) {
#pragma clang fp contract(off)
    float s = u * fN;
    float cf = floorf(s);
    cf = cf > (float)(N - 1) ? (float)(N - 1) : cf;
    w = s - cf;
    int ci = (int)cf;
    return ci < 0 ? 0 : (ci > N - 1 ? N - 1 : ci);
}


template <typename GT> __device__ __forceinline__ void load_row(const GLOBAL GT* p, float v[4]);
template <> __device__ __forceinline__ void load_row<_Float16>(const GLOBAL _Float16* p, float v[4]) {
    const GLOBAL unsigned* q = reinterpret_cast<const GLOBAL unsigned*>(p);
    const unsigned wx = q[0], wy = q[1];
    float2 a = __half22float2(__builtin_bit_cast(__half2, wx)), b = __half22float2(__builtin_bit_cast(__half2, wy));
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
template <> __device__ __forceinline__ void load_row<float>(const GLOBAL float* p, float v[4]) {
    v[0] = p[0]; v[1] = p[1]; v[2] = p[2]; v[3] = p[3];
}

// Lookup t of lane half `half`: table, cell and weights.
template <int L>
__device__ __forceinline__ void lookup_geom(const float u[3][3], int half, int t, const TrainArgs& A, int64_t& base,
                                            int32_t& sy, int64_t& sz, float w[3]) {
    constexpr int NL = 3 * L / 2;
    const int k = half ? NL + t : t;
    const int e = k / L, l = k % L;
    const int N = A.res[l];
    int c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float ue = e == 0 ? u[0][a] : (e == 1 ? u[1][a] : u[2][a]);
        c[a] = cell_coord_t(ue, (float)N, N, w[a]);
    }
    const int32_t N1 = N + 1;
    base = A.toff[k] + (int64_t)((c[2] * N1 + c[1]) * N1 + c[0]) * kFeats;
    sy = N1 * kFeats;
    sz = (int64_t)sy * N1;
}

__global__ void fill_zero_kernel(uint32_t* p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

// Global-address-space atomics: generic (flat) atomics would also wait on the
// LDS counter.  The chunk of 64 latents holding the pair is flagged dirty with a
// plain byte store (no read, no atomic): the Adam pass visits dirty chunks only.
constexpr int kChunkShift = 6;  // latents per dirty flag: 64
__device__ __forceinline__ void add_and_mark(float* p, uint8_t* dirty, int64_t el, float s0, float s1) {
    GLOBAL float* gp = (GLOBAL float*)p;
    if (s0 != 0.0f) __builtin_amdgcn_global_atomic_fadd_f32(gp, s0);
    if (s1 != 0.0f) __builtin_amdgcn_global_atomic_fadd_f32(gp + 1, s1);
    if (s0 != 0.0f || s1 != 0.0f) ((GLOBAL uint8_t*)dirty)[el >> kChunkShift] = 1;
}

// Coarse-level latent gradients are summed per block in an LDS hash table
// before they reach memory.  A coarse table has few vertices, and every wave
// of the batch adds into the same ones: same-address atomics from thousands
// of waves serialise in the L2 (on MI355X the coarse levels' atomics took
// about 70 % of a 262,144-ray step).  The table holds up to kAggSlots vertices (key = element
// index / 2 of the vertex's first latent, values = the two latents' sums) of
// the block's object; a vertex that finds no slot within kAggProbe probes, or
// a query of another object, goes to global atomics directly.  The block adds
// its table to the gradient once, after its last tile.
constexpr int kAggBits = 12;
constexpr int kAggSlots = 1 << kAggBits;
constexpr int kAggProbe = 16;
constexpr int kAggMaxRes = 128;  // levels of at most this many cells per axis are aggregated
constexpr uint32_t kAggEmpty = 0xffffffffu;

__device__ __forceinline__ bool agg_add(uint32_t* keys, float* v0, float* v1, uint32_t key, float s0, float s1) {
    const uint32_t h = (key * 2654435761u) >> (32 - kAggBits);
    for (int p = 0; p < kAggProbe; ++p) {
        const uint32_t slot = (h + (uint32_t)p) & (kAggSlots - 1);
        uint32_t cur = keys[slot];
        if (cur == kAggEmpty) {
            cur = atomicCAS(&keys[slot], kAggEmpty, key);
            if (cur == kAggEmpty) cur = key;
        }
        if (cur == key) {
            atomicAdd(&v0[slot], s0);
            atomicAdd(&v1[slot], s1);
            return true;
        }
    }
    return false;
}

// ---------------------------------------------------------------------------
// T1
// ---------------------------------------------------------------------------
template <int L, typename GT>
__global__ __launch_bounds__(kBlock) void train_fb_kernel(TrainArgs A) {
    constexpr int KH1 = 3 * L;  // local layer-1 inputs per half
    constexpr int NL = 3 * L / 2;
    constexpr int PK1 = KH1 * 4 / 16;  // forward layer-1 packets per M-tile (binary32)
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int half = lane >> 5;
    const int qlane = lane & 31;
    const int H = A.hidden;
    const int64_t n = A.n;
    __shared__ uint32_t agg_key[kAggSlots];
    __shared__ float agg_v0[kAggSlots], agg_v1[kAggSlots];
    for (int i = threadIdx.x; i < kAggSlots; i += kBlock) {
        agg_key[i] = kAggEmpty;
        agg_v0[i] = 0.0f;
        agg_v1[i] = 0.0f;
    }
    // a contiguous range of tiles per block: ordered queries, so the block's
    // coarse cells repeat; its object is that of its first query
    const int64_t tiles = (n + kQueriesPerBlock - 1) / kQueriesPerBlock;
    const int64_t t_begin = (int64_t)blockIdx.x * tiles / gridDim.x;
    const int64_t t_end = (int64_t)(blockIdx.x + 1) * tiles / gridDim.x;
    int32_t agg_obj = -1;
    if (t_begin < t_end) {
        const int64_t s0 = t_begin * kQueriesPerBlock;
        const int64_t q0 = A.perm ? (int64_t)A.perm[s0] : s0;
        const int32_t id0 = A.ids[q0];
        if (id0 >= 0 && id0 < A.num_objects && A.objs[id0].mlp == A.mlp) agg_obj = id0;
    }
    __syncthreads();

    for (int64_t tile = t_begin; tile < t_end; ++tile) {
        const int64_t slot = tile * kQueriesPerBlock + wave * kQueriesPerWave + qlane;
        const bool inb = slot < n;
        const int64_t q = inb && A.perm ? (int64_t)A.perm[slot] : slot;
        float o[3] = {0, 0, 0}, d[3] = {1, 0, 0};
        float tm = 0.0f;
        int32_t id = -1;
        if (inb) {
            const float* r = A.rays + q * 6;
#pragma unroll
            for (int a = 0; a < 3; ++a) { o[a] = r[a]; d[a] = r[3 + a]; }
            tm = A.tmax[q];
            id = A.ids[q];
        }
        bool active = false;
        float u[3][3];
        ObjDev ob{};
        float seg_a = 0.0f, seg_b = 0.0f;
        if (inb && valid_query(o, d, tm, id, A.num_objects)) {
            ob = A.objs[id];
            active = ob.mlp == A.mlp && clip_normalise(o, d, tm, ob, u, seg_a, seg_b) == 1;
        }
        // depth mode: a query takes part only with a target, a finite closest
        // hit and a segment of non-zero length
        float s_tgt = 0.0f;
        if (active && A.t_hit) {
#pragma clang fp contract(off)
            const float th = A.t_hit[q];
            const float span = seg_b - seg_a;
            const bool has = isfinite(th) && span > 0.0f;
            if (has) {
                const float sv = (th - seg_a) / span;
                s_tgt = sv > 0.0f ? (sv < 1.0f ? sv : 1.0f) : 0.0f;
            }
            active = has;
        }
        // ---- encode
        float x[KH1];
#pragma unroll
        for (int c = 0; c < KH1; ++c) x[c] = 0.0f;
        if (active) {
            const GLOBAL GT* grid = (const GLOBAL GT*)ob.grid;
#pragma unroll
            for (int t = 0; t < NL; ++t) {
                int64_t base;
                int32_t sy;
                int64_t sz;
                float w[3];
                lookup_geom<L>(u, half, t, A, base, sy, sz, w);
                float r0[4], r1[4], r2[4], r3[4];
                load_row<GT>(grid + base, r0);
                load_row<GT>(grid + base + sy, r1);
                load_row<GT>(grid + base + sz, r2);
                load_row<GT>(grid + base + sz + sy, r3);
                // corner weights prod (b_a ? w_a : 1 - w_a), formed as ((x y) z), and the
                // sum over corners b = bx + 2 by + 4 bz in that order
                const float x0 = 1.0f - w[0], y0 = 1.0f - w[1], z0 = 1.0f - w[2];
                const float a00 = x0 * y0, a10 = w[0] * y0, a01 = x0 * w[1], a11 = w[0] * w[1];
                const float cw[8] = {a00 * z0, a10 * z0, a01 * z0, a11 * z0, a00 * w[2], a10 * w[2], a01 * w[2], a11 * w[2]};
                const float* rows[4] = {r0, r1, r2, r3};
#pragma unroll
                for (int f = 0; f < kFeats; ++f) {
                    float acc = cw[0] * r0[f];
#pragma unroll
                    for (int cidx = 1; cidx < 8; ++cidx) acc = fmaf(cw[cidx], rows[cidx >> 1][2 * (cidx & 1) + f], acc);
                    x[2 * t + f] = acc;
                }
            }
        }
        if (half == 0) {
            const uint64_t m = __ballot(active);
            if (lane == 0) atomicAdd(A.count, (unsigned)__popcll(m));
        }
        // layer-1 inputs: feature half*KH1 + c, slot
        if (inb) {
#pragma unroll
            for (int c = 0; c < KH1; ++c) A.act[(int64_t)(half * KH1 + c) * n + slot] = x[c];
        }
        // ---- forward, binary32 MFMA (same chain as the query kernel)
        f32x16 acc[2];
        uint32_t mask[kMaxHidden];
        {
            acc[0] = f32x16{};
            acc[1] = f32x16{};
            const float* L1 = A.fwd + A.pack.layer_off[0] / 4;
#pragma unroll
            for (int p = 0; p < PK1; ++p) {
#pragma unroll
                for (int mt = 0; mt < 2; ++mt) {
                    const f32x4 af = load4(L1 + ((mt * PK1 + p) * 64 + lane) * 4);
#pragma unroll
                    for (int qq = 0; qq < 4; ++qq)
                        acc[mt] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[qq], x[4 * p + qq], acc[mt], 0, 0, 0);
                }
            }
        }
        float h[32];
        for (int j = 0; j < H; ++j) {
            // activations of layer j+1 (1-based): relu, mask, store as input of the next layer
            uint32_t mk = 0;
#pragma unroll
            for (int c = 0; c < 32; ++c) {
                const float v = acc[c / 16][c % 16];
                mk |= (v > 0.0f ? 1u : 0u) << c;
                h[c] = v > 0.0f ? v : 0.0f;
            }
            mask[j] = mk;
            if (inb) {
                float* dst = A.act + A.act_off[j + 1];
#pragma unroll
                for (int c = 0; c < 32; ++c) dst[(int64_t)acc_feature(half, c) * n + slot] = h[c];
            }
            if (j + 1 == H) break;
            const float* Lj = A.fwd + A.pack.layer_off[j + 1] / 4;
            acc[0] = f32x16{};
            acc[1] = f32x16{};
#pragma unroll
            for (int p = 0; p < 8; ++p) {
#pragma unroll
                for (int mt = 0; mt < 2; ++mt) {
                    const f32x4 af = load4(Lj + ((mt * 8 + p) * 64 + lane) * 4);
#pragma unroll
                    for (int qq = 0; qq < 4; ++qq)
                        acc[mt] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[qq], h[4 * p + qq], acc[mt], 0, 0, 0);
                }
            }
        }
        // ---- output, loss, dL/dz (unscaled)
        const float* wo = A.fwd + A.pack.layer_off[H] / 4 + half * 32;
        float zp = 0.0f;
#pragma unroll
        for (int c = 0; c < 32; ++c) zp = fmaf(wo[c], h[c], zp);
        const float z = zp + __shfl_xor(zp, 32);
        float dz = 0.0f, lterm = 0.0f;
        if (active) {
            const float sg = 1.0f / (1.0f + expf(-z));
            if (A.grad_y) {
                dz = A.grad_y[q] * (sg * (1.0f - sg));
            } else if (A.t_hit) {  // L2 on the normalised depth: d/dz (y - s)^2 = 2 (y - s) y (1 - y)
                const float e = sg - s_tgt;
                dz = 2.0f * e * (sg * (1.0f - sg));
                lterm = e * e;
            } else {
                const float t = A.labels[q] ? 1.0f : 0.0f;
                dz = sg - t;
                lterm = fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z))) - t * z;
            }
        }
        if (inb && half == 0) A.dz[slot] = dz;
        {
            float ls = half == 0 ? lterm : 0.0f;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) ls += __shfl_xor(ls, off);
            if (lane == 0 && ls != 0.0f) atomicAdd(A.loss_sum, ls);
        }
        // ---- backward: delta_H = w_out * dz * [a_H > 0]
        float dl[32];
#pragma unroll
        for (int c = 0; c < 32; ++c) dl[c] = ((mask[H - 1] >> c) & 1u) ? wo[c] * dz : 0.0f;
        for (int j = H - 1; j >= 0; --j) {
            if (inb) {
                float* dst = A.delta + A.delta_off[j];
#pragma unroll
                for (int c = 0; c < 32; ++c) dst[(int64_t)acc_feature(half, c) * n + slot] = dl[c];
            }
            const float* Bj = A.bwd + (int64_t)j * (2 * 8 * 64 * 4);
            acc[0] = f32x16{};
            acc[1] = f32x16{};
#pragma unroll
            for (int p = 0; p < 8; ++p) {
#pragma unroll
                for (int mt = 0; mt < 2; ++mt) {
                    const f32x4 af = load4(Bj + ((mt * 8 + p) * 64 + lane) * 4);
#pragma unroll
                    for (int qq = 0; qq < 4; ++qq)
                        acc[mt] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[qq], dl[4 * p + qq], acc[mt], 0, 0, 0);
                }
            }
            if (j > 0) {
#pragma unroll
                for (int c = 0; c < 32; ++c) dl[c] = ((mask[j - 1] >> c) & 1u) ? acc[c / 16][c % 16] : 0.0f;
            }
        }
        // acc now holds g_x for this half's local features c = 16 mt + r < KH1
        // ---- scatter into the grid gradient; mark touched vertices
        if (!__ballot(active)) continue;  // wave-uniform
        float* gg = active ? A.grid_grad[id] : nullptr;
        uint8_t* tb = active ? A.touched[id] : nullptr;
        const bool agg_ok = active && id == agg_obj;
#pragma unroll
        for (int t = 0; t < NL; ++t) {
            int64_t base;
            int32_t sy;
            int64_t sz;
            float w[3];
            lookup_geom<L>(u, half, t, A, base, sy, sz, w);
            const float g0 = acc[(2 * t) / 16][(2 * t) % 16], g1 = acc[(2 * t + 1) / 16][(2 * t + 1) % 16];
            const int k = half ? NL + t : t;
            const bool coarse = A.res[k % L] <= kAggMaxRes;
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const int bx = b & 1, by = (b >> 1) & 1, bz = b >> 2;
                const float wt = (bx ? w[0] : 1.0f - w[0]) * (by ? w[1] : 1.0f - w[1]) * (bz ? w[2] : 1.0f - w[2]);
                const int64_t el = base + (bz ? sz : 0) + (by ? sy : 0) + bx * kFeats;
                const float s0 = wt * g0, s1 = wt * g1;
                if (!active || (s0 == 0.0f && s1 == 0.0f)) continue;
                if (coarse && agg_ok && agg_add(agg_key, agg_v0, agg_v1, (uint32_t)(el >> 1), s0, s1)) continue;
                add_and_mark(gg + el, tb, el, s0, s1);
            }
        }
    }
    // the block's coarse-level sums into the object's gradient
    __syncthreads();
    if (agg_obj >= 0) {
        float* gg = A.grid_grad[agg_obj];
        uint8_t* tb = A.touched[agg_obj];
        for (int i = threadIdx.x; i < kAggSlots; i += kBlock) {
            const uint32_t key = agg_key[i];
            if (key == kAggEmpty) continue;
            const int64_t el = (int64_t)key << 1;
            add_and_mark(gg + el, tb, el, agg_v0[i], agg_v1[i]);
        }
    }
}

// ---------------------------------------------------------------------------
// T2: dW partials.  blockIdx.y = layer (0..H-1 hidden layers, H = output row).
// dW_j = D_j X_j^T over the chunk's slots: D_j the layer's output deltas
// (64 x slots, or the 1 x slots dz row), X_j its inputs (kin x slots), both
// [feature][slot] in the workspace.  The block stages kDwStep slots of every
// row of D_j and X_j in LDS with coalesced row loads, then each wave owns one
// 32x32 tile (mt, nt) of the [out][in] gradient and runs its binary32 MFMAs
// from LDS, slots in ascending order.
// ---------------------------------------------------------------------------
constexpr int kDwStep = 64;             // slots per LDS stage
constexpr int kDwLd = kDwStep + 1;      // padded row: lanes reading one slot of 32 rows hit 32 banks
__global__ __launch_bounds__(256) void train_dw_kernel(TrainArgs A) {
    __shared__ float sD[kWidth * kDwLd];
    __shared__ float sX[kWidth * kDwLd];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int mt = wave >> 1, nt = wave & 1;
    const int j = blockIdx.y;
    const int H = A.hidden;
    const int64_t n = A.n;
    const int64_t s0 = (int64_t)blockIdx.x * A.dw_chunk;
    const int64_t s1 = s0 + A.dw_chunk < n ? s0 + A.dw_chunk : n;
    // rows: output deltas of layer j (or dz for the output row); columns: inputs of layer j
    const int kin = j == 0 ? A.din : kWidth;
    const float* D = j < H ? A.delta + A.delta_off[j] : A.dz;
    const int rows = j < H ? kWidth : 1;
    const int cols = j < H ? kin : kWidth;
    const float* X = A.act + A.act_off[j < H ? j : H];
    const int ro = 32 * mt + (lane & 31), co = 32 * nt + (lane & 31);
    const bool live = !(j == H && mt == 1) && !(nt == 1 && cols <= 32);
    f32x16 acc = f32x16{};
    for (int64_t b0 = s0; b0 < s1; b0 += kDwStep) {
        const int cnt = (int)(s1 - b0 < kDwStep ? s1 - b0 : kDwStep);
        __syncthreads();
        // stage: thread t loads slots (t % 64) of rows t / 64, t / 64 + 4, ...; zeros past the chunk
        for (int r = threadIdx.x >> 6; r < kWidth; r += 4) {
            const int sl = threadIdx.x & 63;
            const bool in = sl < cnt;
            sD[r * kDwLd + sl] = in && r < rows ? D[(int64_t)r * n + b0 + sl] : 0.0f;
            sX[r * kDwLd + sl] = in && r < cols ? X[(int64_t)r * n + b0 + sl] : 0.0f;
        }
        __syncthreads();
        if (live) {
            // K-step k takes slots 2k (lane half 0) and 2k + 1 (half 1)
#pragma unroll 8
            for (int k = 0; k < kDwStep / 2; ++k) {
                const int sl = 2 * k + (lane >> 5);
                const float a = sD[ro * kDwLd + sl];
                const float bv = sX[co * kDwLd + sl];
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bv, acc, 0, 0, 0);
            }
        }
    }
    // partial tile -> partials[chunk][param]
    float* out = A.dw_part + (int64_t)blockIdx.x * A.P;
    const int64_t woff = j < H ? A.w_off[j] : A.w_off[H];
    const int ld = j < H ? kin : kWidth;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int orow = 32 * mt + 8 * (r / 4) + 4 * (lane >> 5) + (r % 4);
        const int icol = 32 * nt + (lane & 31);
        const bool ok = j < H ? (orow < kWidth && icol < kin) : (orow == 0 && icol < kWidth && mt == 0);
        if (ok) out[woff + (int64_t)orow * ld + icol] = acc[r];
    }
}

__global__ void train_dw_reduce_kernel(TrainArgs A, int64_t chunks) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < A.P; k += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.0f;
        for (int64_t c = 0; c < chunks; ++c) s += A.dw_part[c * A.P + k];
        A.dw[k] = s;
    }
}

// ---------------------------------------------------------------------------
// T3 / T4: Adam (Kingma & Ba, bias-corrected), gradients scaled by 1/B here.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float adam_update(float theta, float g, float& m, float& v, const AdamDev& a) {
    m = a.beta1 * m + (1.0f - a.beta1) * g;
    v = a.beta2 * v + (1.0f - a.beta2) * g * g;
    const float mh = m / a.bc1, vh = v / a.bc2;
    return theta - a.lr * mh / (sqrtf(vh) + a.eps);
}

__global__ void adam_mlp_kernel(TrainArgs A) {
    const unsigned B = *A.count;
    const float inv = B ? 1.0f / (float)B : 0.0f;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < A.P; k += (int64_t)gridDim.x * blockDim.x) {
        const float g = A.dw[k] * inv;
        if (A.grad_out) A.grad_out[k] = g;
        if (B == 0) continue;
        float m = A.mlp_m[k], v = A.mlp_v[k];
        A.master[k] = adam_update(A.master[k], g, m, v, A.adam);
        A.mlp_m[k] = m;
        A.mlp_v[k] = v;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && A.loss_out) *A.loss_out = B ? *A.loss_sum * inv : 0.0f;
}

// Adam on the latents whose gradient is non-zero, gradient and flag cleared.
// A wave reads 64 chunk flags at once (one per lane), then visits the dirty
// chunks among them, one coalesced 64-latent chunk at a time.
template <typename GT>
__global__ void adam_grid_kernel(TrainArgs A, int32_t obj, int64_t elems) {
    const unsigned B = *A.count;
    const float inv = B ? 1.0f / (float)B : 0.0f;
    GLOBAL float* gg = (GLOBAL float*)A.grid_grad[obj];
    GLOBAL float* gm = (GLOBAL float*)A.grid_m[obj];
    GLOBAL float* gv = (GLOBAL float*)A.grid_v[obj];
    GLOBAL uint8_t* dirty = (GLOBAL uint8_t*)A.touched[obj];
    GLOBAL GT* theta = (GLOBAL GT*)A.grids[obj];
    const int lane = threadIdx.x & 63;
    const int64_t chunks = (elems + 63) >> kChunkShift;
    const int64_t groups = (chunks + 63) >> 6;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t gi = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); gi < groups; gi += waves) {
        const int64_t mine = (gi << 6) + lane;
        const bool d = mine < chunks && dirty[mine];
        uint64_t m = __ballot(d);
        if (d) dirty[mine] = 0;
        while (m) {
            const int j = __builtin_ctzll(m);
            m &= m - 1;
            const int64_t el = (((gi << 6) + j) << kChunkShift) + lane;
            if (el >= elems) continue;
            const float graw = gg[el];
            if (graw == 0.0f) continue;  // zero gradient: latent and moments keep their values
            gg[el] = 0.0f;
            float mm = gm[el], vv = gv[el];
            const float th = adam_update((float)theta[el], graw * inv, mm, vv, A.adam);
            gm[el] = mm;
            gv[el] = vv;
            theta[el] = (GT)th;
        }
    }
}

// Gradient-only mode: scale the accumulated latent gradient by 1/B in the dirty
// chunks and clear the flags (the caller owns and clears the gradient).
__global__ void scale_grid_grad_kernel(TrainArgs A, int32_t obj, int64_t elems) {
    const unsigned B = *A.count;
    const float inv = A.grad_y ? 1.0f : B ? 1.0f / (float)B : 0.0f;
    GLOBAL float* gg = (GLOBAL float*)A.grid_grad[obj];
    GLOBAL uint8_t* dirty = (GLOBAL uint8_t*)A.touched[obj];
    const int lane = threadIdx.x & 63;
    const int64_t chunks = (elems + 63) >> kChunkShift;
    const int64_t groups = (chunks + 63) >> 6;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t gi = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); gi < groups; gi += waves) {
        const int64_t mine = (gi << 6) + lane;
        const bool d = mine < chunks && dirty[mine];
        uint64_t m = __ballot(d);
        if (d) dirty[mine] = 0;
        while (m) {
            const int j = __builtin_ctzll(m);
            m &= m - 1;
            const int64_t el = (((gi << 6) + j) << kChunkShift) + lane;
            if (el < elems) gg[el] *= inv;
        }
    }
}

__global__ void mlp_grad_only_kernel(TrainArgs A) {
    const unsigned B = *A.count;
    const float inv = A.grad_y ? 1.0f : B ? 1.0f / (float)B : 0.0f;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < A.P; k += (int64_t)gridDim.x * blockDim.x)
        if (A.grad_out) A.grad_out[k] = A.dw[k] * inv;
    if (blockIdx.x == 0 && threadIdx.x == 0 && A.loss_out) *A.loss_out = B ? *A.loss_sum * inv : 0.0f;
}

// ---------------------------------------------------------------------------
size_t train_workspace_bytes(int64_t n, int din, int hidden, int64_t P, int64_t* chunk_out) {
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const int64_t chunk = 1024;  // dW split-K chunk: 256 chunks (x 5 layers) for a 262,144-ray batch
    const int64_t chunks = (n + chunk - 1) / chunk;
    if (chunk_out) *chunk_out = chunk;
    size_t b = 0;
    b += al((size_t)(din + (int64_t)hidden * kWidth) * n * 4);  // activations (layer inputs + h_H)
    b += al((size_t)hidden * kWidth * n * 4);                   // deltas
    b += al((size_t)n * 4);                                     // dz
    b += al((size_t)chunks * P * 4);                            // dW partials
    b += al((size_t)P * 4);                                     // dW
    b += 256;                                                   // count, loss
    return b;
}

hipError_t launch_train(TrainArgs A, void* ws, const int32_t* obj_of_mlp, int32_t num_obj_of_mlp,
                        const int64_t* elems_per_obj, int grid_dtype, int levels, int num_cus, hipStream_t s) {
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    int64_t chunk;
    train_workspace_bytes(A.n, A.din, A.hidden, A.P, &chunk);
    const int64_t chunks = (A.n + chunk - 1) / chunk;
    uint8_t* p = reinterpret_cast<uint8_t*>(ws);
    A.act = reinterpret_cast<float*>(p);
    A.act_off[0] = 0;
    for (int j = 1; j <= A.hidden; ++j) A.act_off[j] = ((int64_t)A.din + (int64_t)(j - 1) * kWidth) * A.n;
    p += al((size_t)(A.din + (int64_t)A.hidden * kWidth) * A.n * 4);
    A.delta = reinterpret_cast<float*>(p);
    for (int j = 0; j < A.hidden; ++j) A.delta_off[j] = (int64_t)j * kWidth * A.n;
    p += al((size_t)A.hidden * kWidth * A.n * 4);
    A.dz = reinterpret_cast<float*>(p);
    p += al((size_t)A.n * 4);
    A.dw_part = reinterpret_cast<float*>(p);
    p += al((size_t)chunks * A.P * 4);
    A.dw = reinterpret_cast<float*>(p);
    p += al((size_t)A.P * 4);
    A.count = reinterpret_cast<unsigned*>(p);
    A.loss_sum = reinterpret_cast<float*>(p + 4);
    A.dw_chunk = chunk;
    A.w_off[0] = 0;
    for (int j = 1; j <= A.hidden; ++j) A.w_off[j] = (int64_t)kWidth * A.din + (int64_t)(j - 1) * kWidth * kWidth;
    hipLaunchKernelGGL(fill_zero_kernel, dim3(1), dim3(64), 0, s, reinterpret_cast<uint32_t*>(p), 2);
    const int64_t tiles = (A.n + kQueriesPerBlock - 1) / kQueriesPerBlock;
    int64_t blocks = (int64_t)num_cus * 3;  // three blocks of 48 KB of aggregation table per compute unit
    if (blocks > tiles) blocks = tiles;
    if (levels == 8) {
        if (grid_dtype == 1)
            hipLaunchKernelGGL((train_fb_kernel<8, _Float16>), dim3((unsigned)blocks), dim3(kBlock), 0, s, A);
        else
            hipLaunchKernelGGL((train_fb_kernel<8, float>), dim3((unsigned)blocks), dim3(kBlock), 0, s, A);
    } else {
        if (grid_dtype == 1)
            hipLaunchKernelGGL((train_fb_kernel<4, _Float16>), dim3((unsigned)blocks), dim3(kBlock), 0, s, A);
        else
            hipLaunchKernelGGL((train_fb_kernel<4, float>), dim3((unsigned)blocks), dim3(kBlock), 0, s, A);
    }
    hipLaunchKernelGGL(train_dw_kernel, dim3((unsigned)chunks, (unsigned)(A.hidden + 1)), dim3(256), 0, s, A);
    hipLaunchKernelGGL(train_dw_reduce_kernel, dim3((unsigned)((A.P + 255) / 256)), dim3(256), 0, s, A, chunks);
    if (A.apply_adam)
        hipLaunchKernelGGL(adam_mlp_kernel, dim3((unsigned)((A.P + 255) / 256)), dim3(256), 0, s, A);
    else
        hipLaunchKernelGGL(mlp_grad_only_kernel, dim3((unsigned)((A.P + 255) / 256)), dim3(256), 0, s, A);
    for (int i = 0; i < num_obj_of_mlp; ++i) {
        const int32_t k = obj_of_mlp[i];
        const int64_t elems = elems_per_obj[k];
        const int64_t groups = (((elems + 63) >> kChunkShift) + 63) >> 6;  // 64 chunk flags per wave step
        const int64_t cap = (int64_t)num_cus * 32;
        const unsigned gb = (unsigned)((groups + 3) / 4 < cap ? (groups + 3) / 4 : cap);  // 4 waves per block
        if (!A.apply_adam)
            hipLaunchKernelGGL(scale_grid_grad_kernel, dim3(gb), dim3(256), 0, s, A, k, elems);
        else if (grid_dtype == 1)
            hipLaunchKernelGGL(adam_grid_kernel<_Float16>, dim3(gb), dim3(256), 0, s, A, k, elems);
        else
            hipLaunchKernelGGL(adam_grid_kernel<float>, dim3(gb), dim3(256), 0, s, A, k, elems);
    }
    return hipGetLastError();
}

}  // namespace nif
