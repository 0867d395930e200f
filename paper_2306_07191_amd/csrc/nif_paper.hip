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
// q = 0 maps to theta = 0, phi = 0.
__device__ __forceinline__ void sph_uv(const float q[3], float& u, float& v) {
#pragma clang fp contract(off)
    float l2 = q[0] * q[0];
    l2 = l2 + q[1] * q[1];
    l2 = l2 + q[2] * q[2];
    float cz = l2 > 0.0f ? q[2] * rsqrtf(l2) : 1.0f;
    cz = fminf(fmaxf(cz, -1.0f), 1.0f);
    const float theta = acosf(cz), phi = atan2f(q[1], q[0]);
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

}  // namespace nif
