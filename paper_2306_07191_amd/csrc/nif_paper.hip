// The paper's own networks (Fujieda, Kao, Harada, "Neural Intersection
// Function", HPG 2023, Sec. 3.1, Sec. 3.2, Sec. 5 "Architecture", Table 1):
// spherical 2D grids of the position and the direction (plus a 1D distance
// grid for the inner network) and a leaky-ReLU MLP shared by every object,
// on the MFMA MLP of the fused query kernel.
#include <hip/hip_fp16.h>

#include "nif_device.h"
#include "nif_internal.h"
#include "nif_mlp.h"

namespace nif {

constexpr int kOuterR = 256, kOuterN = 3;                               // Table 1
constexpr int kInnerR = 128, kInnerN = 5, kInnerR1 = 128, kInnerN1 = 3;
constexpr float kPi = 3.14159265358979f, kInvPi = 0.318309886183791f, kInv2Pi = 0.159154943091895f;

// (u, v) = (theta / pi, (phi + pi) / (2 pi)) of the direction of q, in [0, 1];
// q = 0 maps to theta = 0, phi = 0 (atan2 of two zeros).
__device__ __forceinline__ void sph_uv(const float q[3], float& u, float& v) {
#pragma clang fp contract(off)
    float rxy2 = q[0] * q[0];
    rxy2 = rxy2 + q[1] * q[1];
    // polar angle as atan2(|q_xy|, q_z): well conditioned near the poles, where
    // arccos of q_z / |q| is not
    const float theta = atan2f(sqrtf(rxy2), q[2]), phi = atan2f(q[1], q[0]);
    u = fminf(fmaxf(theta * kInvPi, 0.0f), 1.0f);
    v = fminf(fmaxf((phi + kPi) * kInv2Pi, 0.0f), 1.0f);
}

// Vertex-aligned cell and weight of u in [0, 1] on R samples.
__device__ __forceinline__ uint32_t grid_cell(float u, int R, float& w) {
#pragma clang fp contract(off)
    const float s = u * (float)(R - 1);
    uint32_t c = (uint32_t)floorf(s);
    c = c < (uint32_t)(R - 2) ? c : (uint32_t)(R - 2);
    w = s - (float)c;
    return c;
}

// Bilinear lookup of N latents on an R x R grid (rows along u).
template <int R, int N>
__device__ __forceinline__ void lookup2d(const GLOBAL _Float16* g, float u, float v, float* out) {
    float wa, wb;
    const uint32_t a = grid_cell(u, R, wa), b = grid_cell(v, R, wb);
    const GLOBAL _Float16* p00 = g + ((size_t)a * R + b) * N;
    const GLOBAL _Float16* p10 = p00 + (size_t)R * N;
    const float w00 = (1.0f - wa) * (1.0f - wb), w10 = wa * (1.0f - wb), w01 = (1.0f - wa) * wb, w11 = wa * wb;
#pragma unroll
    for (int f = 0; f < N; ++f) {
        float x = w00 * (float)p00[f];
        x = fmaf(w10, (float)p10[f], x);
        x = fmaf(w01, (float)p00[N + f], x);
        out[f] = fmaf(w11, (float)p10[N + f], x);
    }
}

// Outer features (half 0: position grid, half 1: direction grid) or inner
// features (the same on the inner grids, plus the distance grid: half 0 keeps
// its latents 0 and 1, half 1 latent 2 and a zero).
template <int NET>
__device__ __forceinline__ void paper_features(const float o[3], const float d[3], float ta, const PaperObj& ob,
                                               int half, float* xin) {
#pragma clang fp contract(off)
    constexpr int R = NET == 0 ? kOuterR : kInnerR, N = NET == 0 ? kOuterN : kInnerN;
    // q = (p - c) / h with p the entry point (outer) or the origin (inner)
    float qv[3], sv[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float p = NET == 0 ? o[a] + ta * d[a] : o[a];
        qv[a] = (p - ob.c[a]) * ob.ih[a];
        sv[a] = half ? d[a] : qv[a];
    }
    float u, v;
    sph_uv(sv, u, v);
    const GLOBAL _Float16* g = (const GLOBAL _Float16*)ob.grid[NET] + (size_t)half * R * R * N;
    lookup2d<R, N>(g, u, v, xin);
    if constexpr (NET == 1) {
        float l2 = qv[0] * qv[0];
        l2 = l2 + qv[1] * qv[1];
        l2 = l2 + qv[2] * qv[2];
        const float r = fminf(sqrtf(l2) / 1.7320508f, 1.0f);
        float w;
        const uint32_t c = grid_cell(r, kInnerR1, w);
        const GLOBAL _Float16* gr = (const GLOBAL _Float16*)ob.grid[NET] + (size_t)2 * R * R * N + c * kInnerN1;
        float rv[kInnerN1];
#pragma unroll
        for (int f = 0; f < kInnerN1; ++f) rv[f] = fmaf(w, (float)gr[kInnerN1 + f], (1.0f - w) * (float)gr[f]);
        xin[N] = half ? rv[2] : rv[0];
        xin[N + 1] = half ? 0.0f : rv[1];
    }
}

// One pass over the queries: each wave runs the outer MLP if any of its
// queries is outer and the inner MLP if any is inner (both images in LDS).
template <int FLAV>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void nif_paper_kernel(PaperArgs A) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    constexpr int KO = kOuterN, KI = kInnerN + 2;  // layer-1 inputs per half (inner padded 13 -> 14)
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int half = lane >> 5;
    const int qlane = lane & 31;
    const int b = blockIdx.x;
    const int lb = (b & 7) * A.xcd_stride + (b >> 3);
    const int64_t t_begin = (int64_t)lb * A.num_tiles / A.tiles_per_block_num;
    const int64_t t_end = (int64_t)(lb + 1) * A.num_tiles / A.tiles_per_block_num;
    if (t_begin >= t_end) return;
    uint8_t* img[2] = {smem, smem + A.pack[0].bytes};
    for (int net = 0; net < 2; ++net) {
        const int nvec = (int)(A.pack[net].bytes / 16);
        for (int i = threadIdx.x; i < nvec; i += kBlock)
            reinterpret_cast<i32x4*>(img[net])[i] = reinterpret_cast<const i32x4*>(A.packed[net])[i];
    }
    __syncthreads();
    for (int64_t tile = t_begin; tile < t_end; ++tile) {
        const int64_t q = tile * kQueriesPerBlock + wave * kQueriesPerWave + qlane;
        const bool inb = q < A.n;
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
        // class: -2 out of range, -1 invalid, 0 miss, 1 outer, 2 inner
        int cls = -2;
        float xin[KI];
#pragma unroll
        for (int c = 0; c < KI; ++c) xin[c] = 0.0f;
        if (inb) {
            const uint32_t err = query_error_bits(o, d, tm, id, A.num_objects);
            if (err) {
                cls = -1;
                if (A.flags) __hip_atomic_fetch_or(A.flags, err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                const PaperObj ob = A.objs[id];
                float ta, tb;
                if (!clip_segment(o, d, tm, ob.lo, ob.hi, ta, tb)) {
                    cls = 0;
                } else {
                    bool inside = true;
#pragma unroll
                    for (int a = 0; a < 3; ++a) inside = inside && o[a] > ob.lo[a] && o[a] < ob.hi[a];
                    cls = inside ? 2 : 1;
                }
                if (cls == 1)
                    paper_features<0>(o, d, ta, ob, half, xin);
                else if (cls == 2)
                    paper_features<1>(o, d, ta, ob, half, xin);
            }
        }
        float z = 0.0f;
        if (__ballot(cls == 1)) {
            float xo[KO];
#pragma unroll
            for (int c = 0; c < KO; ++c) xo[c] = cls == 1 ? xin[c] : 0.0f;
            const float zz = run_mlp<FLAV, KO, 1>(img[0], A.pack[0], A.hidden[0], xo, nullptr, lane);
            if (cls == 1) z = zz;
        }
        if (__ballot(cls == 2)) {
            float xi[KI];
#pragma unroll
            for (int c = 0; c < KI; ++c) xi[c] = cls == 2 ? xin[c] : 0.0f;
            const float zz = run_mlp<FLAV, KI, 1>(img[1], A.pack[1], A.hidden[1], xi, nullptr, lane);
            if (cls == 2) z = zz;
        }
        if (inb && half == 0) {
            float y, zo;
            if (cls > 0) {
                zo = z;
                y = 1.0f / (1.0f + expf(-z));
            } else if (cls == 0) {
                zo = INFINITY;
                y = 1.0f;
            } else {
                zo = NAN;
                y = NAN;
            }
            if (A.vis) A.vis[q] = y;
            if (A.logit) A.logit[q] = zo;
        }
    }
}

template <int FLAV>
static hipError_t launch_paper_t(const PaperArgs& a0, int num_cus, hipStream_t s) {
    PaperArgs a = a0;
    const int64_t tiles = (a.n + kQueriesPerBlock - 1) / kQueriesPerBlock;
    int64_t blocks = (int64_t)num_cus * 8;
    if (blocks > tiles) blocks = tiles;
    blocks = (blocks + 7) / 8 * 8;
    a.num_tiles = (int32_t)tiles;
    a.tiles_per_block_num = (int32_t)blocks;
    a.xcd_stride = (int32_t)(blocks / 8);
    const size_t lds = (size_t)(a.pack[0].bytes + a.pack[1].bytes);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)nif_paper_kernel<FLAV>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((nif_paper_kernel<FLAV>), dim3((unsigned)blocks), dim3(kBlock), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_paper(int flavor, const PaperArgs& a, int num_cus, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    switch (flavor) {
    case kF32: return launch_paper_t<kF32>(a, num_cus, s);
    case kBF16: return launch_paper_t<kBF16>(a, num_cus, s);
    case kF16: return launch_paper_t<kF16>(a, num_cus, s);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Training of the paper's networks (Sec. 5 "Training": L2 loss and Adam; the
// latents are trained with the MLP through back-propagation, Fig. 2).
// Binary32, one thread per query (the paper trains on batches of 2^11 and
// 2^12 rays): forward with the rows of every layer kept in the workspace, then
// the deltas, then the latent gradients scattered with binary32 atomics.
// Sums over the batch are scaled by 1/B (B = the queries of the network's
// class) where they are consumed.
// ---------------------------------------------------------------------------
template <int NET> struct PaperDims;
template <> struct PaperDims<0> { static constexpr int din = 6, width = 64, hidden = 2, N = kOuterN, R = kOuterR; };
template <> struct PaperDims<1> { static constexpr int din = 13, width = 48, hidden = 3, N = kInnerN, R = kInnerR; };
template <int NET> constexpr int paper_params() {
    using D = PaperDims<NET>;
    return D::width * D::din + (D::hidden - 1) * D::width * D::width + D::width;
}

__device__ __forceinline__ float leaky_grad(float h) { return h > 0.0f ? 1.0f : kLeakySlope; }

// Grid coordinates of a query: position (u, v), direction (u, v), distance r.
template <int NET>
__device__ __forceinline__ void paper_coords(const float o[3], const float d[3], float ta, const PaperObj& ob,
                                             float pu[2], float du[2], float& r) {
#pragma clang fp contract(off)
    float qv[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float p = NET == 0 ? o[a] + ta * d[a] : o[a];
        qv[a] = (p - ob.c[a]) * ob.ih[a];
    }
    sph_uv(qv, pu[0], pu[1]);
    sph_uv(d, du[0], du[1]);
    float l2 = qv[0] * qv[0];
    l2 = l2 + qv[1] * qv[1];
    l2 = l2 + qv[2] * qv[2];
    r = fminf(sqrtf(l2) / 1.7320508f, 1.0f);
}

// Class of a query (as in the forward kernel) and its segment start.
__device__ __forceinline__ int paper_class(const float o[3], const float d[3], float tm, int32_t id, int32_t K,
                                           const PaperObj* objs, float& ta) {
    ta = 0.0f;
    if (query_error_bits(o, d, tm, id, K)) return -1;
    const PaperObj& ob = objs[id];
    float tb;
    if (!clip_segment(o, d, tm, ob.lo, ob.hi, ta, tb)) return 0;
    bool inside = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) inside = inside && o[a] > ob.lo[a] && o[a] < ob.hi[a];
    return inside ? 2 : 1;
}

// Four lanes per query (lanes 4t .. 4t + 3 of a 64-thread block hold query
// t), so that a small batch fills four times as many waves: lane s of a query
// computes the outputs k = s, s + 4, ... of every layer. The layer inputs sit
// in registers, the weights and every hidden layer's outputs in LDS (one
// column per query, read by the query's four lanes), and the rows of the
// workspace are only written, for the dW sums.
constexpr int kTrainBlock = 64, kTrainSplit = 4, kTrainQ = kTrainBlock / kTrainSplit;

// The LDS writes of every lane of the wave before the reads that follow.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// out[k] = leaky(sum_i w[k IN + i] in[i]), i ascending, for this lane's k.
template <int IN, int W>
__device__ __forceinline__ void paper_train_layer(const float* w, const float (&in)[W], float* col, float* row,
                                                  int sub) {
    for (int k = sub; k < W; k += kTrainSplit) {
        float a = 0.0f;
#pragma unroll
        for (int i = 0; i < IN; ++i) a = fmaf(w[k * IN + i], in[i], a);
        const float h = fmaxf(a, kLeakySlope * a);
        col[k * kTrainQ] = h;
        row[k] = h;
    }
}

template <int W>
__device__ __forceinline__ void paper_train_load(const float* col, float (&v)[W]) {
#pragma unroll
    for (int k = 0; k < W; ++k) v[k] = col[k * kTrainQ];
}

// Adds v[m] to dst + off[m] for every active lane of the wave. Lanes with the
// same dst (rays of one batch towards a small light share direction cells)
// are summed first, by the lowest of them, in lane order, from LDS scratch of
// M x 64 floats: one atomic per group and value instead of one per lane.
// GROUP false: plain atomics (where the cells are spread, the grouping costs
// more than the contention it removes).
template <bool GROUP, int M>
__device__ __forceinline__ void grouped_atomic_add(float* dst, const int (&off)[M], const float (&v)[M],
                                                   float* scratch) {
    if constexpr (!GROUP) {
#pragma unroll
        for (int m = 0; m < M; ++m) atomicAdd(dst + off[m], v[m]);
        return;
    }
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int m = 0; m < M; ++m) scratch[m * 64 + lane] = v[m];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const uint64_t key = (uint64_t)dst;
    const uint32_t klo = (uint32_t)key, khi = (uint32_t)(key >> 32);
    uint64_t todo = __ballot(1), peers = 0;
    while (todo) {
        const int l = __builtin_ctzll(todo);
        const bool same = klo == (uint32_t)__builtin_amdgcn_readlane((int)klo, l) &&
                          khi == (uint32_t)__builtin_amdgcn_readlane((int)khi, l);
        const uint64_t g = __ballot(same);
        if (same) peers = g;
        todo &= ~g;
    }
    if (lane == __builtin_ctzll(peers)) {
        float acc[M];
#pragma unroll
        for (int m = 0; m < M; ++m) acc[m] = v[m];
        for (uint64_t rest = peers & (peers - 1); rest; rest &= rest - 1) {
            const int p = __builtin_ctzll(rest);
#pragma unroll
            for (int m = 0; m < M; ++m) acc[m] += scratch[m * 64 + p];
        }
#pragma unroll
        for (int m = 0; m < M; ++m) atomicAdd(dst + off[m], acc[m]);
    }
}

template <int NET>
__global__ __launch_bounds__(kTrainBlock) void paper_train_kernel(PaperTrainArgs A) {
    using D = PaperDims<NET>;
    constexpr int W = D::width, DI = D::din, H = D::hidden, N = D::N, R = D::R;
    constexpr int P = paper_params<NET>();
    constexpr int S = kTrainSplit;
    __shared__ __attribute__((aligned(16))) float w[P];
    __shared__ float act[H * W * kTrainQ];  // act[(j - 1) W + k][query]: layer j's output k
    static_assert(kTrainBlock == 64 && N * 64 <= H * W * kTrainQ && W % S == 0,
                  "one wave per block; scratch of the adds; whole output groups");
    for (int i = threadIdx.x; i < P; i += kTrainBlock) w[i] = A.w[i];
    __syncthreads();
    const int sub = threadIdx.x % S, ql = threadIdx.x / S;
    const int64_t q = (int64_t)blockIdx.x * kTrainQ + ql;
    if (q >= A.n) return;  // the four lanes of a query leave together
    auto hrow = [&](int j) { return A.ws_h + (j == 0 ? q * DI : A.n * DI + ((int64_t)(j - 1) * A.n + q) * W); };
    auto drow = [&](int j) { return A.ws_d + ((int64_t)(j - 1) * A.n + q) * W; };
    auto col = [&](int j) { return act + (j - 1) * W * kTrainQ + ql; };
    float o[3], d[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        o[a] = A.rays[q * 6 + a];
        d[a] = A.rays[q * 6 + 3 + a];
    }
    const float tm = A.tmax[q];
    const int32_t id = A.ids[q];
    float ta;
    const int cls = paper_class(o, d, tm, id, A.num_objects, A.objs, ta);
    if (cls != NET + 1) {  // not in this network's batch: zero rows
        for (int i = sub; i < DI; i += S) hrow(0)[i] = 0.0f;
        for (int j = 1; j <= H; ++j)
            for (int i = sub; i < W; i += S) hrow(j)[i] = drow(j)[i] = 0.0f;
        if (sub == 0) A.dz[q] = 0.0f;
        return;
    }
    const PaperObj ob = A.objs[id];
    const GLOBAL _Float16* g = (const GLOBAL _Float16*)ob.grid[NET];
    float pu[2], du[2], r;
    paper_coords<NET>(o, d, ta, ob, pu, du, r);
    float x[W];
#pragma unroll
    for (int i = 0; i < W; ++i) x[i] = 0.0f;
    lookup2d<R, N>(g, pu[0], pu[1], x);
    lookup2d<R, N>(g + (size_t)R * R * N, du[0], du[1], x + N);
    if constexpr (NET == 1) {
        float wr;
        const uint32_t c = grid_cell(r, kInnerR1, wr);
        const GLOBAL _Float16* gr = g + (size_t)2 * R * R * N + c * kInnerN1;
#pragma unroll
        for (int f = 0; f < kInnerN1; ++f) x[2 * N + f] = fmaf(wr, (float)gr[kInnerN1 + f], (1.0f - wr) * (float)gr[f]);
    }
#pragma unroll
    for (int i = 0; i < DI; ++i)
        if (i % S == sub) hrow(0)[i] = x[i];
    // forward: layer j's outputs to LDS and to row j of the workspace
    paper_train_layer<DI, W>(w, x, col(1), hrow(1), sub);
    int off = W * DI;
    float v[W];
#pragma unroll
    for (int j = 2; j <= H; ++j) {
        wave_lds_sync();
        paper_train_load<W>(col(j - 1), v);
        paper_train_layer<W, W>(w + off, v, col(j), hrow(j), sub);
        off += W * W;
    }
    wave_lds_sync();
    paper_train_load<W>(col(H), v);  // h_H (every lane of the query forms z)
    float z = 0.0f;
#pragma unroll
    for (int k = 0; k < W; ++k) z = fmaf(w[off + k], v[k], z);
    const float y = 1.0f / (1.0f + expf(-z));
    float dz;
    if (A.grad_y) {  // a given dL/dy: the chain rule through the sigmoid
        dz = A.grad_y[q] * y * (1.0f - y);
    } else {
        const float t = A.labels[q] ? 1.0f : 0.0f;
        if (sub == 0) atomicAdd(A.loss_sum, (y - t) * (y - t));
        dz = 2.0f * (y - t) * y * (1.0f - y);
    }
    if (sub == 0) {
        atomicAdd(A.count, 1u);
        A.dz[q] = dz;
    }
    // deltas, layer H down to 1 (v holds the current layer's delta, whole, in
    // every lane of the query); each layer's delta replaces the layer's
    // outputs in LDS
    {
        float* dH = drow(H);
#pragma unroll
        for (int k = 0; k < W; ++k) {
            v[k] = dz * w[off + k] * leaky_grad(v[k]);
            if (k % S == sub) dH[k] = v[k];
        }
    }
#pragma unroll
    for (int j = H; j >= 2; --j) {
        off -= W * W;
        float* c = col(j - 1);
        float* dprev = drow(j - 1);
        for (int i = sub; i < W; i += S) {
            float b = 0.0f;
#pragma unroll
            for (int k = 0; k < W; ++k) b = fmaf(w[off + k * W + i], v[k], b);
            const float e = b * leaky_grad(c[i * kTrainQ]);
            c[i * kTrainQ] = e;
            dprev[i] = e;
        }
        wave_lds_sync();
        paper_train_load<W>(c, v);
    }
    off -= W * DI;
    float gx[DI];
#pragma unroll
    for (int i = 0; i < DI; ++i) {
        float b = 0.0f;
#pragma unroll
        for (int k = 0; k < W; ++k) b = fmaf(w[off + k * DI + i], v[k], b);
        gx[i] = b;
    }
    // latent gradients: lane s of a query takes bilinear corner s of the
    // position and direction grids (lanes 0 and 1 the two samples of the
    // distance grid); the hidden outputs in LDS are spent, so their space is
    // the scratch of the grouped adds (inner network: rays from one surface
    // share distance and direction cells)
    wave_lds_sync();
    float* gg = A.grid_grad[id];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        float wa, wb;
        const uint32_t a = grid_cell(e ? du[0] : pu[0], R, wa), b = grid_cell(e ? du[1] : pu[1], R, wb);
        const float fa = sub & 1 ? wa : 1.0f - wa, fb = sub & 2 ? wb : 1.0f - wb;
        const float cw = fa * fb;
        float* dst = gg + (size_t)e * R * R * N + ((size_t)(a + (sub & 1)) * R + b + (sub >> 1)) * N;
        float gv[N];
        int go[N];
#pragma unroll
        for (int f = 0; f < N; ++f) {
            gv[f] = cw * gx[e * N + f];
            go[f] = f;
        }
        grouped_atomic_add<NET == 1, N>(dst, go, gv, act);
    }
    if constexpr (NET == 1) {
        if (sub < 2) {
            float wr;
            const uint32_t c = grid_cell(r, kInnerR1, wr);
            float* dst = gg + (size_t)2 * R * R * N + (c + sub) * kInnerN1;
            const float cw = sub ? wr : 1.0f - wr;
            float gv[kInnerN1];
            int go[kInnerN1];
#pragma unroll
            for (int f = 0; f < kInnerN1; ++f) {
                gv[f] = cw * gx[2 * N + f];
                go[f] = f;
            }
            grouped_atomic_add<true, kInnerN1>(dst, go, gv, act);
        }
    }
}

// dW sums: thread = one weight, blockIdx.y = a chunk of the batch.
constexpr int kDwChunk = 64;  // the paper's batches are small: many short chunks fill the chip
template <int NET>
__global__ __launch_bounds__(256) void paper_dw_kernel(PaperTrainArgs A) {
    using D = PaperDims<NET>;
    constexpr int W = D::width, DI = D::din, H = D::hidden;
    constexpr int P = paper_params<NET>();
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    // locate (layer j, row k, column i)
    int j = 1, rem = p, in = DI;
    while (j <= H && rem >= W * in) {
        rem -= W * in;
        ++j;
        in = W;
    }
    const int64_t q0 = (int64_t)blockIdx.y * kDwChunk;
    const int64_t q1 = q0 + kDwChunk < A.n ? q0 + kDwChunk : A.n;
    // s = sum over q in [q0, q1), ascending, of a[q sa] b[q sb]; a full chunk
    // unrolled so that its loads are in flight together
    const float *a, *b;
    int64_t sa, sb;
    if (j <= H) {  // hidden layer j: delta_j[q][k] h_(j-1)[q][i]
        const int k = rem / in, i = rem % in;
        a = A.ws_d + (int64_t)(j - 1) * A.n * W + k;
        b = (j == 1 ? A.ws_h : A.ws_h + A.n * DI + (int64_t)(j - 2) * A.n * W) + i;
        sa = W;
        sb = in;
    } else {  // output row: dz[q] h_H[q][i]
        a = A.dz;
        b = A.ws_h + A.n * DI + (int64_t)(H - 1) * A.n * W + rem;
        sa = 1;
        sb = W;
    }
    float s = 0.0f;
    a += q0 * sa;
    b += q0 * sb;
    const int cnt = (int)(q1 - q0), ia = (int)sa, ib = (int)sb;
    if (cnt == kDwChunk) {
#pragma unroll 16
        for (int t = 0; t < kDwChunk; ++t) s = fmaf(a[t * ia], b[t * ib], s);
    } else {
        for (int t = 0; t < cnt; ++t) s = fmaf(a[t * ia], b[t * ib], s);
    }
    atomicAdd(A.dw + p, s);
}

__global__ void paper_zero_kernel(float* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

__global__ void paper_zero_counters_kernel(float* loss_sum, uint32_t* count) {
    if (threadIdx.x == 0) {
        *loss_sum = 0.0f;
        *count = 0u;
    }
}

__device__ __forceinline__ float paper_adam(float theta, float g, float& m, float& v, const AdamDev& a) {
    m = a.beta1 * m + (1.0f - a.beta1) * g;
    v = a.beta2 * v + (1.0f - a.beta2) * g * g;
    const float mh = m / a.bc1, vh = v / a.bc2;
    return theta - a.lr * mh / (sqrtf(vh) + a.eps);
}

// MLP: scale by 1/B, optional gradient output, dense Adam on the master and
// the matching entry of the 64-wide inference master.
template <int NET>
__global__ void paper_mlp_update_kernel(PaperTrainArgs A) {
    using D = PaperDims<NET>;
    constexpr int W = D::width, DI = D::din, H = D::hidden;
    constexpr int P = paper_params<NET>();
    constexpr int DP = NET == 0 ? 6 : 14;  // padded input width of the inference master
    const unsigned B = *A.count;
    const float inv = A.grad_y ? 1.0f : B ? 1.0f / (float)B : 0.0f;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < P; p += gridDim.x * blockDim.x) {
        const float g = A.dw[p] * inv;
        if (A.grad_out) A.grad_out[p] = g;
        if (!A.use_adam || B == 0) continue;
        float m = A.mlp_m[p], v = A.mlp_v[p];
        const float th = paper_adam(A.w[p], g, m, v, A.adam);
        A.w[p] = th;
        A.mlp_m[p] = m;
        A.mlp_v[p] = v;
        // position in the padded master
        int64_t dst;
        if (p < W * DI) {
            const int k = p / DI, i = p % DI;
            int ip = i;
            if (NET == 1) ip = i < 5 ? i : i < 10 ? i + 2 : i == 10 ? 5 : i == 11 ? 6 : 12;
            dst = (int64_t)k * DP + ip;
        } else if (p < W * DI + (H - 1) * W * W) {
            const int rr = p - W * DI, jj = rr / (W * W), k = (rr % (W * W)) / W, i = rr % W;
            dst = (int64_t)kWidth * DP + (int64_t)jj * kWidth * kWidth + (int64_t)k * kWidth + i;
        } else {
            dst = (int64_t)kWidth * DP + (int64_t)(H - 1) * kWidth * kWidth + (p - W * DI - (H - 1) * W * W);
        }
        if (A.padded) A.padded[dst] = th;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && A.loss_out) *A.loss_out = B ? *A.loss_sum * inv : 0.0f;
}

// Latents of one object: scale by 1/B; with Adam, lazy update of the binary16
// latents whose gradient is non-zero (their gradient then cleared).
__global__ void paper_grid_update_kernel(PaperTrainArgs A, int32_t obj, int64_t elems) {
    const unsigned B = *A.count;
    const float inv = A.grad_y ? 1.0f : B ? 1.0f / (float)B : 0.0f;
    float* gg = A.grid_grad[obj];
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < elems; e += (int64_t)gridDim.x * blockDim.x) {
        const float g = gg[e] * inv;
        if (!A.use_adam) {
            gg[e] = g;
            continue;
        }
        if (g == 0.0f) continue;
        gg[e] = 0.0f;
        float m = A.grid_m[obj][e], v = A.grid_v[obj][e];
        __half* th = reinterpret_cast<__half*>(A.grid[obj]) + e;
        const float nt = paper_adam(__half2float(*th), g, m, v, A.adam);
        A.grid_m[obj][e] = m;
        A.grid_v[obj][e] = v;
        *th = __float2half_rn(nt);
    }
}

static int64_t paper_grid_elems_dev(int network) {
    return network == 0 ? 2LL * kOuterR * kOuterR * kOuterN
                        : 2LL * kInnerR * kInnerR * kInnerN + (int64_t)kInnerR1 * kInnerN1;
}

size_t paper_train_workspace_bytes(int network, int64_t n) {
    const int din = network == 0 ? 6 : 13, W = network == 0 ? 64 : 48, H = network == 0 ? 2 : 3;
    const int P = W * din + (H - 1) * W * W + W;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    return al((size_t)n * (din + (size_t)H * W) * 4) + al((size_t)n * H * W * 4) + al((size_t)n * 4) +
           al((size_t)P * 4) + 256;
}

hipError_t launch_paper_train(int network, PaperTrainArgs a, void* ws, hipStream_t s) {
    const int din = network == 0 ? 6 : 13, W = network == 0 ? 64 : 48, H = network == 0 ? 2 : 3;
    const int P = W * din + (H - 1) * W * W + W;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    uint8_t* p = reinterpret_cast<uint8_t*>(ws);
    a.ws_h = reinterpret_cast<float*>(p);
    p += al((size_t)a.n * (din + (size_t)H * W) * 4);
    a.ws_d = reinterpret_cast<float*>(p);
    p += al((size_t)a.n * H * W * 4);
    a.dz = reinterpret_cast<float*>(p);
    p += al((size_t)a.n * 4);
    a.dw = reinterpret_cast<float*>(p);
    p += al((size_t)P * 4);
    a.loss_sum = reinterpret_cast<float*>(p);
    a.count = reinterpret_cast<uint32_t*>(p + 4);
    hipLaunchKernelGGL(paper_zero_counters_kernel, dim3(1), dim3(64), 0, s, a.loss_sum, a.count);
    hipLaunchKernelGGL(paper_zero_kernel, dim3((P + 255) / 256), dim3(256), 0, s, a.dw, (int64_t)P);
    // the latent gradients of every object are sums over this batch only
    const int64_t ge = paper_grid_elems_dev(network);
    if (a.n > 0) {
        // one wave per block: a 2^11-query batch spreads over 32 compute units
        const unsigned blocks = (unsigned)((a.n + kTrainQ - 1) / kTrainQ);
        if (network == 0)
            hipLaunchKernelGGL(paper_train_kernel<0>, dim3(blocks), dim3(kTrainBlock), 0, s, a);
        else
            hipLaunchKernelGGL(paper_train_kernel<1>, dim3(blocks), dim3(kTrainBlock), 0, s, a);
        const dim3 g2((unsigned)((P + 255) / 256), (unsigned)((a.n + kDwChunk - 1) / kDwChunk));
        if (network == 0)
            hipLaunchKernelGGL(paper_dw_kernel<0>, g2, dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL(paper_dw_kernel<1>, g2, dim3(256), 0, s, a);
    }
    if (network == 0)
        hipLaunchKernelGGL(paper_mlp_update_kernel<0>, dim3((P + 255) / 256), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(paper_mlp_update_kernel<1>, dim3((P + 255) / 256), dim3(256), 0, s, a);
    for (int k = 0; k < a.num_objects; ++k)
        hipLaunchKernelGGL(paper_grid_update_kernel, dim3((unsigned)((ge + 255) / 256 < 2048 ? (ge + 255) / 256 : 2048)),
                           dim3(256), 0, s, a, k, ge);
    return hipGetLastError();
}

// Zero one object's latent gradient (before a step's scatter).
hipError_t launch_paper_zero(float* p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(paper_zero_kernel, dim3((unsigned)((n + 255) / 256 < 2048 ? (n + 255) / 256 : 2048)), dim3(256),
                       0, s, p, n);
    return hipGetLastError();
}

}  // namespace nif
