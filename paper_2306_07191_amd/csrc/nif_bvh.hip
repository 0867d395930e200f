// Plain BVH ray casting on the GPU: exact shadow-ray labels for training
// (Sec. 4.2 trains on ray-object intersection results), the baseline the
// paper compares NIF against (Sec. 6 "Performance Evaluation": BVH ray casting
// of the same shadow rays), and closest-hit distances, the depth targets of
// primary rays (Sec. 7).
//
// Builder (host): binned surface-area heuristic, 16 bins on the axis of
// largest centroid extent, leaves of at most 4 triangles, depth-first node
// order.  Traversal (device): one ray per thread, explicit stack, nearer
// child first; any-hit exits on the first hit with 0 < t < t_max, closest-hit
// keeps the nearest and skips boxes beyond it.
// Ray/triangle test: the watertight algorithm of Woop, Benthin and Wald
// (JCGT 2013) in binary32, double-sided.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/nif.h"
#include "nif_internal.h"

namespace nif {

constexpr int kBvhStack = 96;

struct BNode {
    float lo[3];
    int32_t a;  // inner: left child; leaf: first triangle
    float hi[3];
    int32_t b;  // inner: right child (>= 2); leaf: -count (<= 0)
};

struct Tri {
    float v[9];
};

static void build_bvh(const float* tris, int64_t T, std::vector<BNode>& nodes, std::vector<Tri>& out) {
    std::vector<int32_t> idx(T);
    std::vector<float> cen(3 * T), blo(3 * T), bhi(3 * T);
    for (int64_t k = 0; k < T; ++k) {
        idx[k] = (int32_t)k;
        for (int a = 0; a < 3; ++a) {
            float x0 = tris[9 * k + a], x1 = tris[9 * k + 3 + a], x2 = tris[9 * k + 6 + a];
            blo[3 * k + a] = std::min(x0, std::min(x1, x2));
            bhi[3 * k + a] = std::max(x0, std::max(x1, x2));
            cen[3 * k + a] = 0.5f * (blo[3 * k + a] + bhi[3 * k + a]);
        }
    }
    nodes.clear();
    nodes.reserve(2 * T + 1);
    struct Job { int64_t node, first, count; int depth; };
    std::vector<Job> stack;
    nodes.push_back(BNode{});
    stack.push_back({0, 0, T, 0});
    const int NB = 16;
    while (!stack.empty()) {
        Job j = stack.back();
        stack.pop_back();
        BNode nd{};
        float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        float clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int64_t i = j.first; i < j.first + j.count; ++i) {
            int32_t k = idx[i];
            for (int a = 0; a < 3; ++a) {
                lo[a] = std::min(lo[a], blo[3 * k + a]);
                hi[a] = std::max(hi[a], bhi[3 * k + a]);
                clo[a] = std::min(clo[a], cen[3 * k + a]);
                chi[a] = std::max(chi[a], cen[3 * k + a]);
            }
        }
        for (int a = 0; a < 3; ++a) { nd.lo[a] = lo[a]; nd.hi[a] = hi[a]; }
        int axis = 0;
        for (int a = 1; a < 3; ++a)
            if (chi[a] - clo[a] > chi[axis] - clo[axis]) axis = a;
        int64_t mid = -1;
        if (j.count > 4 && chi[axis] > clo[axis] && j.depth < 60) {
            // binned SAH along `axis` (past depth 60 only balanced median splits,
            // so the depth stays below 60 + log2(n) < kBvhStack)
            int cnt[NB] = {0};
            float bl[NB][3], bh[NB][3];
            for (int b = 0; b < NB; ++b)
                for (int a = 0; a < 3; ++a) { bl[b][a] = INFINITY; bh[b][a] = -INFINITY; }
            const float scale = NB / (chi[axis] - clo[axis]);
            auto bin_of = [&](int32_t k) {
                int b = (int)((cen[3 * k + axis] - clo[axis]) * scale);
                return b < 0 ? 0 : (b >= NB ? NB - 1 : b);
            };
            for (int64_t i = j.first; i < j.first + j.count; ++i) {
                int32_t k = idx[i];
                int b = bin_of(k);
                ++cnt[b];
                for (int a = 0; a < 3; ++a) {
                    bl[b][a] = std::min(bl[b][a], blo[3 * k + a]);
                    bh[b][a] = std::max(bh[b][a], bhi[3 * k + a]);
                }
            }
            auto area = [](const float* l, const float* h) {
                float dx = h[0] - l[0], dy = h[1] - l[1], dz = h[2] - l[2];
                return dx * dy + dy * dz + dz * dx;
            };
            float best = INFINITY;
            int best_split = -1;
            for (int s = 1; s < NB; ++s) {
                float l0[3] = {INFINITY, INFINITY, INFINITY}, h0[3] = {-INFINITY, -INFINITY, -INFINITY};
                float l1[3] = {INFINITY, INFINITY, INFINITY}, h1[3] = {-INFINITY, -INFINITY, -INFINITY};
                int c0 = 0, c1 = 0;
                for (int b = 0; b < NB; ++b) {
                    if (!cnt[b]) continue;
                    float* L = b < s ? l0 : l1;
                    float* Hh = b < s ? h0 : h1;
                    (b < s ? c0 : c1) += cnt[b];
                    for (int a = 0; a < 3; ++a) { L[a] = std::min(L[a], bl[b][a]); Hh[a] = std::max(Hh[a], bh[b][a]); }
                }
                if (!c0 || !c1) continue;
                float cost = c0 * area(l0, h0) + c1 * area(l1, h1);
                if (cost < best) { best = cost; best_split = s; }
            }
            if (best_split > 0) {
                int32_t* p = idx.data() + j.first;
                int32_t* q = std::partition(p, p + j.count, [&](int32_t k) { return bin_of(k) < best_split; });
                mid = q - idx.data();
            }
        }
        if (j.count > 4 && (mid <= j.first || mid >= j.first + j.count)) {
            // no useful SAH split: median by centroid
            int32_t* p = idx.data() + j.first;
            std::nth_element(p, p + j.count / 2, p + j.count,
                             [&](int32_t x, int32_t y) { return cen[3 * x + axis] < cen[3 * y + axis]; });
            mid = j.first + j.count / 2;
        }
        if (j.count <= 4) {
            nd.a = (int32_t)j.first;
            nd.b = -(int32_t)j.count;
            nodes[j.node] = nd;
            continue;
        }
        const int64_t left = (int64_t)nodes.size();
        nodes.push_back(BNode{});
        nodes.push_back(BNode{});
        nd.a = (int32_t)left;
        nd.b = (int32_t)(left + 1);
        nodes[j.node] = nd;
        stack.push_back({left + 1, mid, j.first + j.count - mid, j.depth + 1});
        stack.push_back({left, j.first, mid - j.first, j.depth + 1});
    }
    out.resize(T);
    for (int64_t i = 0; i < T; ++i) memcpy(out[i].v, tris + 9 * (int64_t)idx[i], sizeof(Tri));
}

// ---------------------------------------------------------------------------
__device__ __forceinline__ bool tri_hit(const float* v, const float o[3], const float d[3], int kx, int ky, int kz,
                                        float Sx, float Sy, float Sz, float tmax, float* t_out = nullptr) {
#pragma clang fp contract(off)
    const float Ax = v[0 + kx] - o[kx], Ay = v[0 + ky] - o[ky], Az0 = v[0 + kz] - o[kz];
    const float Bx = v[3 + kx] - o[kx], By = v[3 + ky] - o[ky], Bz0 = v[3 + kz] - o[kz];
    const float Cx = v[6 + kx] - o[kx], Cy = v[6 + ky] - o[ky], Cz0 = v[6 + kz] - o[kz];
    const float ax = Ax - Sx * Az0, ay = Ay - Sy * Az0;
    const float bx = Bx - Sx * Bz0, by = By - Sy * Bz0;
    const float cx = Cx - Sx * Cz0, cy = Cy - Sy * Cz0;
    float U = cx * by - cy * bx;
    float V = ax * cy - ay * cx;
    float W = bx * ay - by * ax;
    if (U == 0.0f || V == 0.0f || W == 0.0f) {  // edge case: redo the edge tests in binary64
        U = (float)((double)cx * by - (double)cy * bx);
        V = (float)((double)ax * cy - (double)ay * cx);
        W = (float)((double)bx * ay - (double)by * ax);
    }
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return false;
    float det = U + V + W;
    if (det == 0.0f) return false;
    float T = U * (Sz * Az0) + V * (Sz * Bz0) + W * (Sz * Cz0);
    if (det < 0.0f) { T = -T; det = -det; }
    if (!(T > 0.0f)) return false;
    if (!(isinf(tmax) || T < tmax * det)) return false;
    if (t_out) *t_out = T / det;
    return true;
}

// CLOSEST = false: any hit, vis[i] = 0 on the first hit with 0 < t < t_max.
// CLOSEST = true: the nearest hit, t_hit[i] = its distance (+inf for none);
// boxes beyond the best hit so far are skipped, nearer child first.
template <bool CLOSEST>
__global__ __launch_bounds__(256) void bvh_trace_kernel(const BNode* __restrict__ nodes, const Tri* __restrict__ tris,
                                                        const float* __restrict__ rays, const float* __restrict__ tmaxv,
                                                        int64_t n, uint8_t* __restrict__ vis, float* __restrict__ t_hit) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float* r = rays + 6 * i;
        const float o[3] = {r[0], r[1], r[2]}, d[3] = {r[3], r[4], r[5]};
        const float tmax = tmaxv[i];
        float inv[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) inv[a] = 1.0f / d[a];
        int kz = fabsf(d[0]) > fabsf(d[1]) ? (fabsf(d[0]) > fabsf(d[2]) ? 0 : 2) : (fabsf(d[1]) > fabsf(d[2]) ? 1 : 2);
        int kx = kz == 2 ? 0 : kz + 1, ky = kx == 2 ? 0 : kx + 1;
        if (d[kz] < 0.0f) { int t = kx; kx = ky; ky = t; }
        const float Sx = d[kx] / d[kz], Sy = d[ky] / d[kz], Sz = 1.0f / d[kz];
        int32_t stack[kBvhStack];
        int sp = 0;
        int32_t node = 0;
        bool hit = false;
        float best = INFINITY;  // closest hit so far
        // slab test widened by a few ulps so that rounding never drops a box the
        // triangle test would hit
        auto box = [&](const BNode& b, float& tn) {
            float t0 = 0.0f, t1 = CLOSEST ? fminf(tmax, best) : tmax;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                float l = (b.lo[a] - o[a]) * inv[a], h = (b.hi[a] - o[a]) * inv[a];
                if (l != l) l = -INFINITY;  // 0 * inf: the ray lies in the slab plane
                if (h != h) h = INFINITY;
                float mn = fminf(l, h), mx = fmaxf(l, h);
                t0 = fmaxf(t0, mn - 2.4e-7f * fabsf(mn));
                t1 = fminf(t1, mx + 2.4e-7f * fabsf(mx));
            }
            tn = t0;
            return t0 <= t1;
        };
        while (true) {
            const BNode nd = nodes[node];
            if (nd.b <= 0) {  // leaf (possibly empty); children always have larger indices
                for (int32_t k = nd.a; k < nd.a - nd.b; ++k) {
                    float t;
                    if (tri_hit(tris[k].v, o, d, kx, ky, kz, Sx, Sy, Sz, tmax, CLOSEST ? &t : nullptr)) {
                        hit = true;
                        if (!CLOSEST) break;
                        best = fminf(best, t);
                    }
                }
                if ((!CLOSEST && hit) || sp == 0) break;
                node = stack[--sp];
                continue;
            }
            float t_l, t_r;
            const bool hl = box(nodes[nd.a], t_l), hr = box(nodes[nd.b], t_r);
            if (hl && hr) {
                const bool lf = t_l <= t_r;
                if (sp < kBvhStack) stack[sp++] = lf ? nd.b : nd.a;
                node = lf ? nd.a : nd.b;
            } else if (hl || hr) {
                node = hl ? nd.a : nd.b;
            } else {
                if (sp == 0) break;
                node = stack[--sp];
            }
        }
        if (CLOSEST) t_hit[i] = best;
        else vis[i] = hit ? 0 : 1;
    }
}

}  // namespace nif

using namespace nif;

struct nif_bvh {
    BNode* d_nodes = nullptr;
    Tri* d_tris = nullptr;
    int64_t num_nodes = 0, num_tris = 0;
};

extern "C" nif_status nif_bvh_create(const float* tris, int64_t num_tris, nif_bvh** out) {
    if (!out || (num_tris > 0 && !tris) || num_tris < 0) return NIF_ERR_INVALID_ARG;
    if (num_tris > ((int64_t)1 << 30)) return NIF_ERR_UNSUPPORTED;
    nif_bvh* h = new (std::nothrow) nif_bvh();
    if (!h) return NIF_ERR_INVALID_ARG;
    std::vector<BNode> nodes;
    std::vector<Tri> sorted;
    if (num_tris > 0) {
        build_bvh(tris, num_tris, nodes, sorted);
    } else {
        BNode empty{};
        for (int a = 0; a < 3; ++a) { empty.lo[a] = INFINITY; empty.hi[a] = -INFINITY; }
        empty.a = 0;
        empty.b = 0;  // leaf with no triangles
        nodes.push_back(empty);
    }
    h->num_nodes = (int64_t)nodes.size();
    h->num_tris = num_tris;
    if (hipMalloc(&h->d_nodes, sizeof(BNode) * nodes.size()) != hipSuccess ||
        hipMemcpy(h->d_nodes, nodes.data(), sizeof(BNode) * nodes.size(), hipMemcpyHostToDevice) != hipSuccess) {
        delete h;
        return NIF_ERR_HIP;
    }
    if (num_tris > 0 &&
        (hipMalloc(&h->d_tris, sizeof(Tri) * sorted.size()) != hipSuccess ||
         hipMemcpy(h->d_tris, sorted.data(), sizeof(Tri) * sorted.size(), hipMemcpyHostToDevice) != hipSuccess)) {
        (void)hipFree(h->d_nodes);
        delete h;
        return NIF_ERR_HIP;
    }
    *out = h;
    return NIF_OK;
}

extern "C" void nif_bvh_destroy(nif_bvh* h) {
    if (!h) return;
    if (h->d_nodes) (void)hipFree(h->d_nodes);
    if (h->d_tris) (void)hipFree(h->d_tris);
    delete h;
}

extern "C" int64_t nif_bvh_num_nodes(const nif_bvh* h) { return h ? h->num_nodes : 0; }

extern "C" nif_status nif_bvh_anyhit(const nif_bvh* h, const float* rays, const float* t_max, int64_t n,
                                     uint8_t* visible, void* stream) {
    if (!h || n < 0) return NIF_ERR_INVALID_ARG;
    if (n == 0) return NIF_OK;
    if (!rays || !t_max || !visible) return NIF_ERR_INVALID_ARG;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(bvh_trace_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, h->d_nodes,
                       h->d_tris, rays, t_max, n, visible, nullptr);
    return hipGetLastError() == hipSuccess ? NIF_OK : NIF_ERR_HIP;
}

extern "C" nif_status nif_bvh_closest(const nif_bvh* h, const float* rays, const float* t_max, int64_t n, float* t_hit,
                                      void* stream) {
    if (!h || n < 0) return NIF_ERR_INVALID_ARG;
    if (n == 0) return NIF_OK;
    if (!rays || !t_max || !t_hit) return NIF_ERR_INVALID_ARG;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(bvh_trace_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, h->d_nodes,
                       h->d_tris, rays, t_max, n, nullptr, t_hit);
    return hipGetLastError() == hipSuccess ? NIF_OK : NIF_ERR_HIP;
}
