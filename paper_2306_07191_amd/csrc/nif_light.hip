// Light importance sampling of shadow-ray directions for training samples
// (Fujieda, Kao, Harada, "Neural Intersection Function", HPG 2023, Sec. 5
// "Training" and Sec. 6 "Comparison of Sampling Method"): a light triangle is
// chosen in proportion to its radiant flux through a tabulated CDF searched by
// bisection, then a uniform point on it; the sample is the shadow ray from a
// shading point to that point.
#include <math.h>

#include <vector>

#include "nif_device.h"
#include "nif_internal.h"

namespace nif {

struct LightTri {
    float v0[3], e1[3], e2[3];  // vertex 0 and the two edges from it
    float n[3];                 // unit normal
    float pa;                   // P(triangle) / area
};

// First entry of tab[0, L) greater than u0 (the last one if none).
__device__ __forceinline__ int32_t cdf_search(const float* tab, int32_t L, float u0) {
    int32_t lo = 0, hi = L - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (tab[mid] > u0)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// Tables of up to this many entries are searched in LDS (64 KB), each
// persistent block reading the table once; larger ones in global memory.
constexpr int32_t kLightLdsEntries = 16384;
constexpr int kLightBlock = 256, kLightLdsBlocks = 1024;

template <bool LDS>
__global__ __launch_bounds__(kLightBlock) void light_sample_kernel(
    const float* __restrict__ tab, const LightTri* __restrict__ tri, int32_t L, const float* __restrict__ points,
    const float* __restrict__ u, int64_t n, float* __restrict__ rays, float* __restrict__ tmax,
    float* __restrict__ pdf, int32_t* __restrict__ which) {
#pragma clang fp contract(off)
    extern __shared__ float stab[];
    if constexpr (LDS) {
        for (int32_t i = threadIdx.x; i < L; i += kLightBlock) stab[i] = tab[i];
        __syncthreads();
    }
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const float u0 = u[3 * k], u1 = u[3 * k + 1], u2 = u[3 * k + 2];
        int32_t lo;
        if constexpr (LDS)
            lo = cdf_search(stab, L, u0);
        else
            lo = cdf_search(tab, L, u0);
        const LightTri t = tri[lo];
        const float su = sqrtf(u1), b1 = 1.0f - su, b2 = u2 * su;
        float x[3], v[3];
        float d2 = 0.0f;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            x[a] = points[3 * k + a];
            const float p = t.v0[a] + b1 * t.e1[a] + b2 * t.e2[a];
            v[a] = p - x[a];
            d2 = d2 + v[a] * v[a];
        }
        const float dist = sqrtf(d2);
        float cs = 0.0f;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float da = v[a] / dist;
            rays[6 * k + a] = x[a];
            rays[6 * k + 3 + a] = da;
            cs = cs + t.n[a] * da;
        }
        tmax[k] = dist;
        if (pdf) pdf[k] = t.pa * d2 / fabsf(cs);
        if (which) which[k] = lo;
    }
}

struct LightTable {
    float* d_tab = nullptr;
    LightTri* d_tri = nullptr;
    int32_t L = 0;
};

// Host tables: flux pi L A in binary64 (cross product e1 x e2 componentwise),
// running sums in order divided by the total, rounded to binary32.
static void build_light(const float* tris, const float* radiance, int64_t L, std::vector<float>& tab,
                        std::vector<LightTri>& out) {
#pragma clang fp contract(off)
    std::vector<double> area((size_t)L), fl((size_t)L);
    out.resize((size_t)L);
    double run = 0.0;
    std::vector<double> runs((size_t)L);
    for (int64_t i = 0; i < L; ++i) {
        const float* t = tris + 9 * i;
        double e1[3], e2[3];
        for (int a = 0; a < 3; ++a) {
            e1[a] = (double)t[3 + a] - (double)t[a];
            e2[a] = (double)t[6 + a] - (double)t[a];
        }
        const double c0 = e1[1] * e2[2] - e1[2] * e2[1];
        const double c1 = e1[2] * e2[0] - e1[0] * e2[2];
        const double c2 = e1[0] * e2[1] - e1[1] * e2[0];
        const double ln = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
        area[(size_t)i] = 0.5 * ln;
        fl[(size_t)i] = M_PI * (double)radiance[i] * area[(size_t)i];
        run += fl[(size_t)i];
        runs[(size_t)i] = run;
        LightTri& o = out[(size_t)i];
        for (int a = 0; a < 3; ++a) {
            o.v0[a] = t[a];
            o.e1[a] = (float)e1[a];
            o.e2[a] = (float)e2[a];
        }
        o.n[0] = (float)(c0 / ln);
        o.n[1] = (float)(c1 / ln);
        o.n[2] = (float)(c2 / ln);
    }
    tab.resize((size_t)L);
    for (int64_t i = 0; i < L; ++i) {
        tab[(size_t)i] = (float)(runs[(size_t)i] / run);
        out[(size_t)i].pa = (float)(fl[(size_t)i] / run / area[(size_t)i]);
    }
    tab[(size_t)L - 1] = 1.0f;
}

hipError_t light_create(const float* tris, const float* radiance, int64_t L, void** out, const char** why) {
    *why = nullptr;
    for (int64_t i = 0; i < L; ++i)
        if (!(radiance[i] >= 0.0f) || !isfinite(radiance[i])) {
            *why = "radiance must be finite and >= 0";
            return hipErrorInvalidValue;
        }
    std::vector<float> tab;
    std::vector<LightTri> tri;
    build_light(tris, radiance, L, tab, tri);
    double total = 0.0;
    for (int64_t i = 0; i < L; ++i) {
        const LightTri& t = tri[(size_t)i];
        if (!isfinite(t.n[0]) || !isfinite(t.n[1]) || !isfinite(t.n[2]) || !isfinite(t.pa)) {
            *why = "degenerate light triangle (zero area)";
            return hipErrorInvalidValue;
        }
        total += t.pa;
    }
    if (!(total > 0.0)) {
        *why = "the lights emit no flux";
        return hipErrorInvalidValue;
    }
    LightTable* lt = new LightTable;
    lt->L = (int32_t)L;
    hipError_t e = hipMalloc(&lt->d_tab, sizeof(float) * L);
    if (e == hipSuccess) e = hipMalloc(&lt->d_tri, sizeof(LightTri) * L);
    if (e == hipSuccess) e = hipMemcpy(lt->d_tab, tab.data(), sizeof(float) * L, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(lt->d_tri, tri.data(), sizeof(LightTri) * L, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (lt->d_tab) (void)hipFree(lt->d_tab);
        if (lt->d_tri) (void)hipFree(lt->d_tri);
        delete lt;
        return e;
    }
    *out = lt;
    return hipSuccess;
}

void light_destroy(void* h) {
    LightTable* lt = reinterpret_cast<LightTable*>(h);
    if (!lt) return;
    (void)hipFree(lt->d_tab);
    (void)hipFree(lt->d_tri);
    delete lt;
}

int32_t light_count(const void* h) { return reinterpret_cast<const LightTable*>(h)->L; }

hipError_t launch_light_sample(const void* h, const float* points, const float* u, int64_t n, float* rays,
                               float* tmax, float* pdf, int32_t* which, hipStream_t s) {
    const LightTable* lt = reinterpret_cast<const LightTable*>(h);
    if (n <= 0) return hipSuccess;
    const int64_t need = (n + kLightBlock - 1) / kLightBlock;
    if (lt->L <= kLightLdsEntries) {
        const int64_t b = need < kLightLdsBlocks ? need : kLightLdsBlocks;
        hipLaunchKernelGGL(light_sample_kernel<true>, dim3((unsigned)b), dim3(kLightBlock),
                           (size_t)lt->L * sizeof(float), s, lt->d_tab, lt->d_tri, lt->L, points, u, n, rays, tmax,
                           pdf, which);
    } else {
        const int64_t b = need < 65536 ? need : 65536;
        hipLaunchKernelGGL(light_sample_kernel<false>, dim3((unsigned)b), dim3(kLightBlock), 0, s, lt->d_tab,
                           lt->d_tri, lt->L, points, u, n, rays, tmax, pdf, which);
    }
    return hipGetLastError();
}

}  // namespace nif
