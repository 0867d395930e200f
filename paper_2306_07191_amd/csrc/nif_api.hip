// Host runtime of libnif.so: the C ABI declared in include/nif.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <stdlib.h>

#include <algorithm>
#include <atomic>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/nif.h"
#include "nif_internal.h"

using namespace nif;

static thread_local std::string g_err;

static nif_status fail(nif_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}
static nif_status ok() {
    g_err.clear();
    return NIF_OK;
}
#define HIP_TRY(expr)                                                                                \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess) return fail(NIF_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

struct ObjHost {
    float aabb[6];
    void* grid = nullptr;
    int32_t mlp = -1;
    bool set = false;
    bool image_built = false;  // its registered query image holds its current grid (nif_build_image, nif_prepare)
    float* grad = nullptr;  // training buffers
    float* m = nullptr;
    float* v = nullptr;
    void* touched = nullptr;  // dirty flag per 64 latents (training)
};

constexpr int kTileRing = 64;  // tile-counter blocks per context for calls without a workspace

struct nif_ctx {
    nif_model_desc d;
    int32_t K, M;
    int32_t din;
    int32_t res[kMaxLevels];
    int64_t toff[3 * kMaxLevels + 1];
    int64_t grid_elems, P;
    std::vector<ObjHost> objs;
    std::vector<float*> masters;
    std::vector<std::vector<float>> fp8;  // per MLP, 2H scales (empty = unset)
    ObjDev* d_objs = nullptr;
    uint8_t* d_packed[4] = {nullptr, nullptr, nullptr, nullptr};
    float* d_scales = nullptr;
    PackInfo pack[4];
    bool prepared[4] = {false, false, false, false};
    int num_cus = 256;
    int device = 0;
    int32_t order_mode = 2;  // NIF_ORDER_AUTO
    int32_t window_sort = 2;  // NIF_OPT_WINDOW_SORT: 2 = when there is no query image
    int32_t tile_shape = 0;   // NIF_OPT_TILE_SHAPE: fused kernel shape outside plans
    int32_t order_bits = -1;  // NIF_OPT_ORDER_BITS: bucket Morton bits per axis at most (-1: automatic)
    std::vector<float*> mlp_m, mlp_v;  // Adam moments per MLP
    // device tables of per-object training pointers: grad, m, v, touched, grid
    void** d_train_tab = nullptr;
    bool train_tab_dirty = true;
    uint8_t* d_train_fwd = nullptr;  // binary32 forward image of the MLP being trained
    float* d_train_bwd = nullptr;    // backward image
    // query images of binary16 grids (NIF_OPT_GRID_IMAGE), caller-owned buffers
    int32_t image_mode = 0;
    int64_t ioff[3 * kMaxLevels + 1];
    std::vector<void*> images;  // per object, registered by nif_set_image, built by nif_prepare
    bool images_ready = false;
    // bumped by every change that a captured plan cannot follow (image mode,
    // object table, option changes); a plan refuses to launch once it differs
    uint64_t epoch = 1;
    uint32_t* d_flags = nullptr;  // domain-error bits of queries (nif_get_error_flags)
    // tile counters of fused-query calls that bring no workspace: a ring of
    // kTileRing blocks, one per call in turn
    uint8_t* d_tile_ring = nullptr;
    std::atomic<uint32_t> tile_ring_next{0};
    uint8_t* d_tree = nullptr;  // box tree of the pair expansion (cluster boxes, member boxes, member ids)
    PairTree tree{};
};

// Host side of the pair expansion's box tree (see PairTree): the flat layout
// of its boxes and ids, and its root box.
struct PairTreeHost {
    std::vector<float> cbox, mbox;
    std::vector<int32_t> mid;
    int32_t C = 0;
    float root[6];
};

static PairTreeHost build_pair_tree(const std::vector<ObjDev>& od) {
    PairTreeHost t;
    const int K = (int)od.size();
    for (int a = 0; a < 3; ++a) {
        t.root[a] = INFINITY;
        t.root[3 + a] = -INFINITY;
        for (const ObjDev& o : od) {
            t.root[a] = fminf(t.root[a], o.lo[a]);
            t.root[3 + a] = fmaxf(t.root[3 + a], o.hi[a]);
        }
    }
    std::vector<int> order(K);
    for (int k = 0; k < K; ++k) order[k] = k;
    if (K > 64) {  // clusters: runs of 64 in the Morton order of the box centres (10 bits per axis)
        float slo[3], shi[3];
        for (int a = 0; a < 3; ++a) {
            slo[a] = INFINITY;
            shi[a] = -INFINITY;
            for (const ObjDev& o : od) {
                slo[a] = fminf(slo[a], 0.5f * (o.lo[a] + o.hi[a]));
                shi[a] = fmaxf(shi[a], 0.5f * (o.lo[a] + o.hi[a]));
            }
        }
        auto spread = [](uint64_t v) {
            uint64_t r = 0;
            for (int b = 0; b < 10; ++b) r |= ((v >> b) & 1ull) << (3 * b);
            return r;
        };
        std::vector<std::pair<uint64_t, int>> key(K);
        for (int k = 0; k < K; ++k) {
            uint64_t m = 0;
            for (int a = 0; a < 3; ++a) {
                const float ext = shi[a] - slo[a];
                const float u = ext > 0.0f ? (0.5f * (od[k].lo[a] + od[k].hi[a]) - slo[a]) / ext : 0.0f;
                const uint64_t q = (uint64_t)fminf(fmaxf(u * 1023.0f, 0.0f), 1023.0f);
                m |= spread(q) << a;
            }
            key[k] = {m, k};
        }
        std::sort(key.begin(), key.end());
        for (int k = 0; k < K; ++k) order[k] = key[k].second;
    }
    t.C = (K + 63) / 64;
    t.mbox.assign((size_t)t.C * 64 * 6, 0.0f);
    t.mid.assign((size_t)t.C * 64, -1);
    t.cbox.assign((size_t)t.C * 6, 0.0f);
    for (int c = 0; c < t.C; ++c) {
        float* cb = &t.cbox[(size_t)c * 6];
        for (int a = 0; a < 3; ++a) {
            cb[a] = INFINITY;
            cb[3 + a] = -INFINITY;
        }
        for (int j = 0; j < 64; ++j) {
            const int i = c * 64 + j;
            float* mb = &t.mbox[(size_t)i * 6];
            if (i >= K) {
                for (int a = 0; a < 3; ++a) {
                    mb[a] = INFINITY;
                    mb[3 + a] = -INFINITY;
                }
                continue;
            }
            const ObjDev& o = od[order[i]];
            t.mid[i] = order[i];
            for (int a = 0; a < 3; ++a) {
                mb[a] = o.lo[a];
                mb[3 + a] = o.hi[a];
                cb[a] = fminf(cb[a], o.lo[a]);
                cb[3 + a] = fmaxf(cb[3 + a], o.hi[a]);
            }
        }
    }
    return t;
}

static void drop_images(nif_ctx* c) {
    c->images.assign(c->K, nullptr);
    c->images_ready = false;
    for (ObjHost& o : c->objs) o.image_built = false;
}

// Offsets of the 3 L tables inside one object's query image.
static void image_offsets(nif_ctx* c) {
    int64_t o = 0;
    for (int k = 0; k < 3 * c->d.levels; ++k) {
        c->ioff[k] = o;
        o += image_table_elems(c->res[k % c->d.levels], c->image_mode);
    }
    c->ioff[3 * c->d.levels] = o;
}

// Objects answered from their query image alone (no grid) cannot be trained
// or read through their grid.
static nif_status require_grids(const nif_ctx* c, const char* where) {
    for (int k = 0; k < c->K; ++k)
        if (c->objs[k].set && !c->objs[k].grid)
            return fail(NIF_ERR_STATE, "%s: object %d has no grid (it is answered from its query image)", where, k);
    return NIF_OK;
}

// Elements of one object's query image for image kind `mode` (0: none).
static int64_t image_elems(const nif_ctx* c, int32_t mode) {
    if (mode == 0) return 0;
    int64_t o = 0;
    for (int k = 0; k < 3 * c->d.levels; ++k) o += image_table_elems(c->res[k % c->d.levels], mode);
    return o;
}

// Whether the ordering also sorts every 4,096-query window by the fine key.
static bool window_sorted(const nif_ctx* c) {
    return c->window_sort == 2 ? c->image_mode == 0 : c->window_sort == 1;
}

static bool uses_order(const nif_ctx* c, int64_t n) {
    if (c->order_mode == 0) return false;
    if (c->order_mode == 1) return true;
    return n >= 65536;
}

extern "C" const char* nif_last_error(void) { return g_err.c_str(); }
extern "C" const char* nif_version(void) { return "nif-mi355x 0.1 (gfx950)"; }

// ---------------------------------------------------------------------------
// level resolutions: rounded geometric progression res_min .. res_max
// ---------------------------------------------------------------------------
static void level_resolutions(const nif_model_desc& d, int32_t* res) {
    for (int l = 0; l < d.levels; ++l) {
        if (d.levels == 1) {
            res[l] = d.res_min;
            continue;
        }
        double r = d.res_min * pow((double)d.res_max / d.res_min, (double)l / (d.levels - 1));
        res[l] = (int32_t)floor(r + 0.5);
    }
}

extern "C" nif_status nif_create(const nif_model_desc* desc, int32_t num_objects, int32_t num_mlps, nif_ctx** out) {
    if (!desc || !out) return fail(NIF_ERR_INVALID_ARG, "nif_create: NULL argument");
    const nif_model_desc& d = *desc;
    if (num_objects < 1 || num_mlps < 1) return fail(NIF_ERR_INVALID_ARG, "nif_create: need >= 1 object and MLP");
    if (num_objects > 4096) return fail(NIF_ERR_UNSUPPORTED, "nif_create: at most 4096 objects");
    if (d.feats != kFeats) return fail(NIF_ERR_UNSUPPORTED, "feats must be %d", kFeats);
    if (d.width != kWidth) return fail(NIF_ERR_UNSUPPORTED, "width must be %d", kWidth);
    if (d.levels != 4 && d.levels != 8) return fail(NIF_ERR_UNSUPPORTED, "levels must be 4 or 8");
    if (d.hidden_layers < 1 || d.hidden_layers > kMaxHidden)
        return fail(NIF_ERR_UNSUPPORTED, "hidden_layers must be in [1, %d]", kMaxHidden);
    if (d.res_min < 1 || d.res_max < d.res_min || d.res_max > 1024)
        return fail(NIF_ERR_UNSUPPORTED, "need 1 <= res_min <= res_max <= 1024");
    if (d.grid_dtype != NIF_F32 && d.grid_dtype != NIF_F16)
        return fail(NIF_ERR_UNSUPPORTED, "grid_dtype must be NIF_F32 or NIF_F16");
    nif_ctx* c = new (std::nothrow) nif_ctx();
    if (!c) return fail(NIF_ERR_INVALID_ARG, "out of host memory");
    c->d = d;
    c->K = num_objects;
    c->M = num_mlps;
    c->din = 3 * d.levels * d.feats;
    level_resolutions(d, c->res);
    int64_t o = 0;
    for (int e = 0; e < 3; ++e)
        for (int l = 0; l < d.levels; ++l) {
            c->toff[e * d.levels + l] = o;
            const int64_t n1 = c->res[l] + 1;
            o += n1 * n1 * n1 * d.feats;
        }
    c->toff[3 * d.levels] = o;
    c->grid_elems = o;
    c->P = (int64_t)d.width * c->din + (int64_t)(d.hidden_layers - 1) * d.width * d.width + d.width;
    c->image_mode = 0;
    c->images.assign(num_objects, nullptr);
    c->objs.resize(num_objects);
    c->masters.assign(num_mlps, nullptr);
    c->fp8.resize(num_mlps);
    c->mlp_m.assign(num_mlps, nullptr);
    c->mlp_v.assign(num_mlps, nullptr);
    if (hipGetDevice(&c->device) == hipSuccess) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) == hipSuccess && cus > 0)
            c->num_cus = cus;
    }
    for (int f = 0; f < 4; ++f) c->pack[f] = pack_info(f, c->din, d.hidden_layers);
    *out = c;
    return ok();
}

extern "C" void nif_destroy(nif_ctx* c) {
    if (!c) return;
    if (c->d_objs) (void)hipFree(c->d_objs);
    for (auto& p : c->d_packed)
        if (p) (void)hipFree(p);
    if (c->d_scales) (void)hipFree(c->d_scales);
    if (c->d_train_tab) (void)hipFree(c->d_train_tab);
    if (c->d_train_fwd) (void)hipFree(c->d_train_fwd);
    if (c->d_train_bwd) (void)hipFree(c->d_train_bwd);
    if (c->d_flags) (void)hipFree(c->d_flags);
    if (c->d_tile_ring) (void)hipFree(c->d_tile_ring);
    if (c->d_tree) (void)hipFree(c->d_tree);
    delete c;
}

extern "C" nif_status nif_param_layout(const nif_ctx* c, int64_t* grid_elems, int64_t* table_offsets,
                                       int32_t* level_res, int64_t* mlp_params) {
    if (!c) return fail(NIF_ERR_INVALID_ARG, "nif_param_layout: NULL context");
    if (grid_elems) *grid_elems = c->grid_elems;
    if (table_offsets) memcpy(table_offsets, c->toff, sizeof(int64_t) * (3 * c->d.levels + 1));
    if (level_res) memcpy(level_res, c->res, sizeof(int32_t) * c->d.levels);
    if (mlp_params) *mlp_params = c->P;
    return ok();
}

static void invalidate(nif_ctx* c) {
    for (bool& p : c->prepared) p = false;
}

extern "C" nif_status nif_set_object(nif_ctx* c, int32_t obj, const float* aabb, void* grid, int32_t mlp_index) {
    if (!c || !aabb) return fail(NIF_ERR_INVALID_ARG, "nif_set_object: NULL argument");
    if (obj < 0 || obj >= c->K) return fail(NIF_ERR_INVALID_ARG, "object %d out of range [0, %d)", obj, c->K);
    if (!grid && !(c->image_mode && c->images[obj] && c->objs[obj].image_built))
        return fail(NIF_ERR_STATE, "nif_set_object: object %d has no built query image to answer from without a grid",
                    obj);
    if (mlp_index < 0 || mlp_index >= c->M) return fail(NIF_ERR_INVALID_ARG, "mlp %d out of range", mlp_index);
    for (int a = 0; a < 3; ++a) {
        if (!isfinite(aabb[a]) || !isfinite(aabb[3 + a]) || !(aabb[3 + a] > aabb[a]))
            return fail(NIF_ERR_INVALID_ARG, "object %d: AABB must be finite with hi > lo on every axis", obj);
    }
    ObjHost& o = c->objs[obj];
    memcpy(o.aabb, aabb, sizeof o.aabb);
    if (grid) o.image_built = false;  // a grid given again: the image is rebuilt from it
    o.grid = grid;
    o.mlp = mlp_index;
    o.set = true;
    invalidate(c);
    ++c->epoch;
    return ok();
}

extern "C" nif_status nif_set_mlp(nif_ctx* c, int32_t mlp, float* weights) {
    if (!c || !weights) return fail(NIF_ERR_INVALID_ARG, "nif_set_mlp: NULL argument");
    if (mlp < 0 || mlp >= c->M) return fail(NIF_ERR_INVALID_ARG, "mlp %d out of range", mlp);
    c->masters[mlp] = weights;
    invalidate(c);
    return ok();
}

extern "C" nif_status nif_set_fp8_scales(nif_ctx* c, int32_t mlp, const float* scales) {
    if (!c || !scales) return fail(NIF_ERR_INVALID_ARG, "nif_set_fp8_scales: NULL argument");
    if (mlp < 0 || mlp >= c->M) return fail(NIF_ERR_INVALID_ARG, "mlp %d out of range", mlp);
    const int H = c->d.hidden_layers;
    for (int i = 0; i < 2 * H; ++i)
        if (!isfinite(scales[i]) || !(scales[i] > 0.0f)) return fail(NIF_ERR_INVALID_ARG, "scales must be > 0");
    c->fp8[mlp].assign(scales, scales + 2 * H);
    c->prepared[kFP8] = false;
    return ok();
}

extern "C" nif_status nif_init_grid(nif_ctx* c, int32_t obj, uint64_t seed, float amp, void* stream) {
    if (!c) return fail(NIF_ERR_INVALID_ARG, "nif_init_grid: NULL context");
    if (obj < 0 || obj >= c->K || !c->objs[obj].set)
        return fail(NIF_ERR_INVALID_ARG, "object %d not registered", obj);
    if (!c->objs[obj].grid) return fail(NIF_ERR_STATE, "nif_init_grid: object %d has no grid", obj);
    if (!isfinite(amp) || amp < 0.0f) return fail(NIF_ERR_INVALID_ARG, "amp must be finite and >= 0");
    HIP_TRY(launch_init_grid(c->objs[obj].grid, c->d.grid_dtype, c->grid_elems, seed, (uint64_t)obj, amp,
                             (hipStream_t)stream));
    return ok();
}

extern "C" nif_status nif_prepare(nif_ctx* c, int32_t dtype, void* stream) {
    if (!c) return fail(NIF_ERR_INVALID_ARG, "nif_prepare: NULL context");
    if (dtype < 0 || dtype > 3) return fail(NIF_ERR_UNSUPPORTED, "unknown dtype %d", dtype);
    for (int k = 0; k < c->K; ++k)
        if (!c->objs[k].set) return fail(NIF_ERR_STATE, "object %d not registered", k);
    for (int m = 0; m < c->M; ++m) {
        if (!c->masters[m]) return fail(NIF_ERR_STATE, "MLP %d not registered", m);
        if (dtype == NIF_FP8_E4M3 && c->fp8[m].empty()) return fail(NIF_ERR_STATE, "MLP %d has no FP8 scales", m);
    }
    if (c->image_mode)
        for (int k = 0; k < c->K; ++k)
            if (!c->images[k])
                return fail(NIF_ERR_STATE, "object %d has no query image buffer (nif_image_bytes, nif_set_image)", k);
    for (int k = 0; k < c->K; ++k)
        if (!c->objs[k].grid && !(c->image_mode && c->objs[k].image_built))
            return fail(NIF_ERR_STATE, "object %d has neither a grid nor a built query image", k);
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipStreamSynchronize(s));
    if (!c->d_flags) {
        HIP_TRY(hipMalloc(&c->d_flags, 256));
        HIP_TRY(launch_fill_u32(c->d_flags, 1, 0u, s));
    }
    if (!c->d_tile_ring) {  // zero once, on the stream of the weights; every launch on a block leaves it zero
        HIP_TRY(hipMalloc(&c->d_tile_ring, kTileRing * kTileCtrBytes));
        HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(c->d_tile_ring), (int64_t)(kTileRing * kTileCtrBytes / 4),
                                0u, s));
    }
    // query images of the grids, in the caller's buffers (rebuilt on every
    // call: the grids may have changed; an object without a grid keeps the
    // image built from its last grid)
    if (c->image_mode) {
        image_offsets(c);
        for (int k = 0; k < c->K; ++k) {
            if (!c->objs[k].grid) continue;
            HIP_TRY(launch_build_image(c->objs[k].grid, c->images[k], c->toff, c->ioff, c->res, c->d.levels,
                                       c->image_mode, s));
            c->objs[k].image_built = true;
        }
        c->images_ready = true;
    }
    // object table
    std::vector<ObjDev> od(c->K);
    for (int k = 0; k < c->K; ++k) {
        const ObjHost& o = c->objs[k];
        for (int a = 0; a < 3; ++a) {
            od[k].lo[a] = o.aabb[a];
            od[k].hi[a] = o.aabb[3 + a];
            od[k].ext[a] = o.aabb[3 + a] - o.aabb[a];
        }
        od[k].mlp = o.mlp;
        od[k].grid = o.grid;
        od[k].image = c->image_mode ? c->images[k] : nullptr;
    }
    if (!c->d_objs) HIP_TRY(hipMalloc(&c->d_objs, sizeof(ObjDev) * c->K));
    HIP_TRY(hipMemcpy(c->d_objs, od.data(), sizeof(ObjDev) * c->K, hipMemcpyHostToDevice));
    {  // the pair expansion's box tree: cluster boxes, member boxes, member ids, one buffer
        const PairTreeHost t = build_pair_tree(od);
        const size_t nc = t.cbox.size() * 4, nm = t.mbox.size() * 4, ni = t.mid.size() * 4;
        if (!c->d_tree) HIP_TRY(hipMalloc(&c->d_tree, nc + nm + ni));
        HIP_TRY(hipMemcpy(c->d_tree, t.cbox.data(), nc, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(c->d_tree + nc, t.mbox.data(), nm, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(c->d_tree + nc + nm, t.mid.data(), ni, hipMemcpyHostToDevice));
        c->tree.cbox = reinterpret_cast<const float*>(c->d_tree);
        c->tree.mbox = reinterpret_cast<const float*>(c->d_tree + nc);
        c->tree.mid = reinterpret_cast<const int32_t*>(c->d_tree + nc + nm);
        c->tree.C = t.C;
        for (int a = 0; a < 6; ++a) c->tree.root[a] = t.root[a];
    }
    // weights, packed on the device from the binary32 masters
    const int flav = dtype;
    const PackInfo& P = c->pack[flav];
    if (!c->d_packed[flav]) HIP_TRY(hipMalloc(&c->d_packed[flav], (size_t)P.bytes * c->M));
    if (flav == kFP8) {
        const int H = c->d.hidden_layers;
        std::vector<float> sc((size_t)2 * H * c->M);
        for (int m = 0; m < c->M; ++m) memcpy(&sc[(size_t)2 * H * m], c->fp8[m].data(), sizeof(float) * 2 * H);
        if (!c->d_scales) HIP_TRY(hipMalloc(&c->d_scales, sizeof(float) * sc.size()));
        HIP_TRY(hipMemcpy(c->d_scales, sc.data(), sizeof(float) * sc.size(), hipMemcpyHostToDevice));
    }
    for (int m = 0; m < c->M; ++m)
        HIP_TRY(launch_pack_forward(c->masters[m], c->d_packed[flav] + (int64_t)m * P.bytes, P, flav, c->din,
                                    c->d.width, flav == kFP8 ? c->d_scales + (int64_t)2 * c->d.hidden_layers * m : nullptr,
                                    s));
    c->prepared[flav] = true;
    return ok();
}

static size_t train_bytes(const nif_ctx* c, int64_t n);

// Ordering workspace, the queries as 32-byte records, then the fused query's
// tile counters (the ordering layout is a multiple of 256 bytes).
static size_t order_packed_bytes(const nif_ctx* c, int64_t n) {
    return order_workspace_bytes(n, c->K) + ((size_t)n * 32 + 255) / 256 * 256 + kTileCtrBytes;
}
static float4* records_in(const nif_ctx* c, void* ws, int64_t n) {
    return reinterpret_cast<float4*>(reinterpret_cast<uint8_t*>(ws) + order_workspace_bytes(n, c->K));
}
static uint32_t* tile_ctr_in(const nif_ctx* c, void* ws, int64_t n) {
    return reinterpret_cast<uint32_t*>(reinterpret_cast<uint8_t*>(ws) + order_workspace_bytes(n, c->K) +
                                       ((size_t)n * 32 + 255) / 256 * 256);
}

extern "C" size_t nif_workspace_bytes(const nif_ctx* c, int64_t n, int32_t mode) {
    if (!c || n < 0) return 0;
    if (mode == 2) return calib_workspace_bytes(n, c->din);  // also n = 0: the maxima words
    if (n == 0) return 0;
    if (mode == 1) return train_bytes(c, n);
    return uses_order(c, n) ? order_packed_bytes(c, n) : 0;
}

extern "C" nif_status nif_set_option(nif_ctx* c, int32_t option, int64_t value) {
    if (!c) return fail(NIF_ERR_INVALID_ARG, "nif_set_option: NULL context");
    switch (option) {
    case NIF_OPT_ORDER:
        if (value < 0 || value > 2) return fail(NIF_ERR_INVALID_ARG, "NIF_OPT_ORDER takes 0, 1 or 2");
        c->order_mode = (int32_t)value;
        return ok();
    case NIF_OPT_WINDOW_SORT:
        if (value < 0 || value > 2) return fail(NIF_ERR_INVALID_ARG, "NIF_OPT_WINDOW_SORT takes 0, 1 or 2");
        c->window_sort = (int32_t)value;
        return ok();
    case NIF_OPT_ORDER_BITS:
        if (value < -1 || value > 4) return fail(NIF_ERR_INVALID_ARG, "NIF_OPT_ORDER_BITS takes -1 to 4");
        c->order_bits = (int32_t)value;
        return ok();
    case NIF_OPT_TILE_SHAPE:
        if (value < 0 || value > 2) return fail(NIF_ERR_INVALID_ARG, "NIF_OPT_TILE_SHAPE takes 0, 1 or 2");
        c->tile_shape = (int32_t)value;
        return ok();
    case NIF_OPT_GRID_IMAGE:
        if (value < 0 || value > 2) return fail(NIF_ERR_INVALID_ARG, "NIF_OPT_GRID_IMAGE takes 0, 1 or 2");
        if (value > 0 && c->d.grid_dtype != NIF_F16)
            return fail(NIF_ERR_UNSUPPORTED, "NIF_OPT_GRID_IMAGE needs binary16 grids");
        if ((int32_t)value != c->image_mode) {
            drop_images(c);  // sizes differ between kinds: the caller registers new buffers
            c->image_mode = (int32_t)value;
            for (bool& p : c->prepared) p = false;
            ++c->epoch;
        }
        return ok();
    }
    return fail(NIF_ERR_INVALID_ARG, "unknown option %d", option);
}

extern "C" size_t nif_image_bytes(const nif_ctx* c) {
    if (!c) return 0;
    return (size_t)image_elems(c, c->image_mode) * 2;
}

extern "C" nif_status nif_set_image(nif_ctx* c, int32_t obj, void* image, size_t bytes) {
    if (!c) return fail(NIF_ERR_INVALID_ARG, "nif_set_image: NULL context");
    if (obj < 0 || obj >= c->K) return fail(NIF_ERR_INVALID_ARG, "object %d out of range [0, %d)", obj, c->K);
    if (c->image_mode == 0) return fail(NIF_ERR_STATE, "nif_set_image: NIF_OPT_GRID_IMAGE is 0");
    if (!image) return fail(NIF_ERR_INVALID_ARG, "nif_set_image: NULL image");
    if (reinterpret_cast<uintptr_t>(image) % 256 != 0)
        return fail(NIF_ERR_INVALID_ARG, "nif_set_image: image must be 256-byte aligned");
    const size_t need = nif_image_bytes(c);
    if (bytes < need) return fail(NIF_ERR_WORKSPACE, "nif_set_image: need %zu bytes", need);
    if (c->images[obj] != image) {
        c->images[obj] = image;
        c->images_ready = false;
        c->objs[obj].image_built = false;
        for (bool& p : c->prepared) p = false;
        ++c->epoch;
    }
    return ok();
}

extern "C" nif_status nif_build_image(nif_ctx* c, int32_t obj, void* stream) {
    if (!c) return fail(NIF_ERR_INVALID_ARG, "nif_build_image: NULL context");
    if (obj < 0 || obj >= c->K || !c->objs[obj].set)
        return fail(NIF_ERR_INVALID_ARG, "nif_build_image: object %d not registered", obj);
    if (c->image_mode == 0) return fail(NIF_ERR_STATE, "nif_build_image: NIF_OPT_GRID_IMAGE is 0");
    if (!c->images[obj]) return fail(NIF_ERR_STATE, "nif_build_image: object %d has no image buffer", obj);
    if (!c->objs[obj].grid) return fail(NIF_ERR_STATE, "nif_build_image: object %d has no grid", obj);
    image_offsets(c);
    HIP_TRY(launch_build_image(c->objs[obj].grid, c->images[obj], c->toff, c->ioff, c->res, c->d.levels,
                               c->image_mode, (hipStream_t)stream));
    c->objs[obj].image_built = true;
    return ok();
}

static nif_status check_query_args(nif_ctx* c, int32_t dtype, const void* rays, const void* ids, const void* tmax,
                                   int64_t n, const void* vis, const char* where) {
    if (!c) return fail(NIF_ERR_INVALID_ARG, "%s: NULL context", where);
    if (n < 0) return fail(NIF_ERR_INVALID_ARG, "%s: n < 0", where);
    if (dtype < 0 || dtype > 3) return fail(NIF_ERR_UNSUPPORTED, "unknown dtype %d", dtype);
    if (n == 0) return NIF_OK;
    if (!rays || !ids || !tmax || !vis) return fail(NIF_ERR_INVALID_ARG, "%s: NULL input or output", where);
    if (n > ((int64_t)1 << 32) - 1) return fail(NIF_ERR_UNSUPPORTED, "%s: n must be below 2^32", where);
    return NIF_OK;
}

// The fused query.  tile_ctr: the launch's tile counters from the caller's
// workspace (ctr_zero: the ordering pass before it zeroed them), or null for
// the next block of the context's ring (zero between launches).
static nif_status run_query(nif_ctx* c, int32_t dtype, const float* rays, const int32_t* ids, const float* tmax,
                            const uint32_t* perm, int64_t n, float* vis, float* logits, hipStream_t s,
                            int32_t blocks_per_cu = 0, const float4* qrec = nullptr, int32_t shape = -1,
                            uint32_t* tile_ctr = nullptr, bool ctr_zero = false) {
    FwdArgs a{};
    if (!tile_ctr) {
        if (!c->d_tile_ring) return fail(NIF_ERR_STATE, "context not prepared");
        const uint32_t slot = c->tile_ring_next.fetch_add(1, std::memory_order_relaxed) % kTileRing;
        tile_ctr = reinterpret_cast<uint32_t*>(c->d_tile_ring + (size_t)slot * kTileCtrBytes);
        ctr_zero = true;
    }
    a.tile_ctr = tile_ctr;
    a.tile_ctr_reset = ctr_zero ? 1 : 0;
    a.qrec = qrec;
    a.shape = shape >= 0 ? shape : c->tile_shape;
    a.flags = c->d_flags;
    a.blocks_per_cu = blocks_per_cu;
    a.use_image = c->images_ready ? c->image_mode : 0;
    for (int k = 0; k < 3 * c->d.levels; ++k) a.ioff[k] = c->ioff[k];
    a.perm = perm;
    a.rays = rays;
    a.ids = ids;
    a.tmax = tmax;
    a.n = n;
    a.vis = vis;
    a.logit = logits;
    a.objs = c->d_objs;
    a.num_objects = c->K;
    a.hidden = c->d.hidden_layers;
    a.packed = c->d_packed[dtype];
    a.pack = c->pack[dtype];
    a.fp8_scales = dtype == kFP8 ? c->d_scales : nullptr;
    for (int k = 0; k < 3 * c->d.levels; ++k) a.toff[k] = c->toff[k];
    for (int l = 0; l < c->d.levels; ++l) a.res[l] = c->res[l];
    HIP_TRY(launch_forward(dtype, c->d.levels, c->d.grid_dtype, a, c->num_cus, s));
    return ok();
}

// max_bits: the bucket key's Morton bits per axis at most (-1 automatic);
// kOrderBitsOption: the context's NIF_OPT_ORDER_BITS.
constexpr int32_t kOrderBitsOption = -2;
static nif_status run_order(nif_ctx* c, const float* rays, const int32_t* ids, const float* tmax, int64_t n,
                            uint32_t* perm_dst, void* ws, const uint32_t** perm, hipStream_t s,
                            bool refine = true, float4* qrec = nullptr, uint32_t* zero_words = nullptr,
                            int32_t max_bits = kOrderBitsOption) {
    OrderArgs o{};
    o.zero_words = zero_words;
    o.qrec = qrec;
    o.no_refine = refine ? 0 : 1;
    o.rays = rays;
    o.ids = ids;
    o.tmax = tmax;
    o.n = n;
    o.objs = c->d_objs;
    o.num_objects = c->K;
    o.max_bits = max_bits == kOrderBitsOption ? c->order_bits : max_bits;
    o.perm = perm_dst;
    HIP_TRY(launch_order(o, ws, s, perm));
    return ok();
}

// The query after argument checks: ordering into ws (need > 0 bytes of it,
// nothing in it has to start at zero), then the fused kernel.
static nif_status query_in(nif_ctx* c, int32_t dtype, const float* rays, const int32_t* ids, const float* tmax,
                           int64_t n, float* vis, float* logits, void* ws, size_t need, void* stream) {
    nif_status st = NIF_OK;
    const uint32_t* perm = nullptr;
    float4* qrec = nullptr;
    uint32_t* ctr = nullptr;
    if (need > 0) {
        qrec = records_in(c, ws, n);
        ctr = tile_ctr_in(c, ws, n);
        st = run_order(c, rays, ids, tmax, n, nullptr, ws, &perm, (hipStream_t)stream, window_sorted(c), qrec, ctr);
        if (st != NIF_OK) return st;
    }
    return run_query(c, dtype, rays, ids, tmax, perm, n, vis, logits, (hipStream_t)stream, 0, qrec, -1, ctr,
                     ctr != nullptr);
}

extern "C" nif_status nif_query(nif_ctx* c, int32_t dtype, const float* rays, const int32_t* ids, const float* tmax,
                                int64_t n, float* vis, float* logits, void* ws, size_t ws_bytes, void* stream) {
    nif_status st = check_query_args(c, dtype, rays, ids, tmax, n, vis, "nif_query");
    if (st != NIF_OK || n == 0) return st == NIF_OK ? ok() : st;
    const size_t need = nif_workspace_bytes(c, n, 0);
    if (ws_bytes < need || (need > 0 && !ws)) return fail(NIF_ERR_WORKSPACE, "workspace too small: need %zu bytes", need);
    if (!c->prepared[dtype]) return fail(NIF_ERR_STATE, "context not prepared for dtype %d", dtype);
    return query_in(c, dtype, rays, ids, tmax, n, vis, logits, ws, need, stream);
}

// Scratch of nif_query_noalloc: the ordering workspace and the 32-byte query
// records, in a static device array instead of a caller workspace.  Every GPU
// the library runs on holds its own copy at its own address; the host-side
// name `scratch` is not that address, so the address is looked up once per
// device and only the looked-up pointer is handed to kernels.
static __device__ __align__(256) uint8_t scratch[NIF_QUERY_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxScratchDevices] = {};

static nif_status scratch_of_current_device(void** out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxScratchDevices)
        return fail(NIF_ERR_UNSUPPORTED, "nif_query_noalloc: device %d beyond the %d supported", dev,
                    kMaxScratchDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(NIF_ERR_HIP, "nif_query_noalloc: no device address for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return NIF_OK;
}

extern "C" nif_status nif_query_noalloc(nif_ctx* c, int32_t dtype, const float* rays, const int32_t* ids,
                                        const float* tmax, int64_t n, float* vis, float* logits, void* stream) {
    nif_status st = check_query_args(c, dtype, rays, ids, tmax, n, vis, "nif_query_noalloc");
    if (st != NIF_OK || n == 0) return st == NIF_OK ? ok() : st;
    const size_t need = nif_workspace_bytes(c, n, 0);
    if (need > (size_t)NIF_QUERY_NOALLOC_SCRATCH_BYTES)
        return fail(NIF_ERR_UNSUPPORTED,
                    "nif_query_noalloc: %lld queries need %zu bytes of scratch, the library holds %zu; "
                    "use nif_query with a workspace or split the batch",
                    (long long)n, need, (size_t)NIF_QUERY_NOALLOC_SCRATCH_BYTES);
    if (!c->prepared[dtype]) return fail(NIF_ERR_STATE, "context not prepared for dtype %d", dtype);
    void* ws = nullptr;
    if (need > 0) {
        st = scratch_of_current_device(&ws);
        if (st != NIF_OK) return st;
    }
    return query_in(c, dtype, rays, ids, tmax, n, vis, logits, ws, need, stream);
}

extern "C" size_t nif_order_workspace_bytes(const nif_ctx* c, int64_t n) {
    if (!c || n <= 0) return 0;
    return order_workspace_bytes(n, c->K);
}

extern "C" nif_status nif_order(nif_ctx* c, const float* rays, const int32_t* ids, const float* tmax, int64_t n,
                                uint32_t* perm, void* ws, size_t ws_bytes, void* stream) {
    nif_status st = check_query_args(c, 0, rays, ids, tmax, n, perm, "nif_order");
    if (st != NIF_OK || n == 0) return st == NIF_OK ? ok() : st;
    const size_t need = order_workspace_bytes(n, c->K);
    if (ws_bytes < need || !ws) return fail(NIF_ERR_WORKSPACE, "workspace too small: need %zu bytes", need);
    if (!c->d_objs) return fail(NIF_ERR_STATE, "context not prepared");
    const uint32_t* p = nullptr;
    return run_order(c, rays, ids, tmax, n, perm, ws, &p, (hipStream_t)stream, window_sorted(c));
}

extern "C" nif_status nif_order_keys(nif_ctx* c, const uint32_t* keys, int64_t n, uint32_t* perm, void* ws,
                                     size_t ws_bytes, void* stream) {
    if (!c) return fail(NIF_ERR_INVALID_ARG, "nif_order_keys: NULL context");
    if (n < 0) return fail(NIF_ERR_INVALID_ARG, "nif_order_keys: negative size");
    if (n == 0) return ok();
    if (!keys || !perm) return fail(NIF_ERR_INVALID_ARG, "nif_order_keys: NULL keys or perm");
    if (n > ((int64_t)1 << 32) - 1) return fail(NIF_ERR_UNSUPPORTED, "nif_order_keys: n must be below 2^32");
    const size_t need = order_workspace_bytes(n, c->K);
    if (ws_bytes < need || !ws) return fail(NIF_ERR_WORKSPACE, "workspace too small: need %zu bytes", need);
    if (!c->d_objs) return fail(NIF_ERR_STATE, "context not prepared");
    OrderArgs o{};
    o.key_in = keys;
    o.max_bits = c->order_bits;
    o.no_refine = window_sorted(c) ? 0 : 1;
    o.n = n;
    o.objs = c->d_objs;
    o.num_objects = c->K;
    o.perm = perm;
    const uint32_t* p = nullptr;
    HIP_TRY(launch_order(o, ws, (hipStream_t)stream, &p));
    return ok();
}

extern "C" nif_status nif_order_packed(nif_ctx* c, const float* rays, const int32_t* ids, const float* tmax,
                                       int64_t n, uint32_t* perm, float* packed, void* ws, size_t ws_bytes,
                                       void* stream) {
    nif_status st = check_query_args(c, 0, rays, ids, tmax, n, perm, "nif_order_packed");
    if (st != NIF_OK || n == 0) return st == NIF_OK ? ok() : st;
    if (!packed) return fail(NIF_ERR_INVALID_ARG, "nif_order_packed: NULL packed");
    if (reinterpret_cast<uintptr_t>(packed) % 16 != 0)
        return fail(NIF_ERR_INVALID_ARG, "nif_order_packed: packed must be 16-byte aligned");
    const size_t need = order_workspace_bytes(n, c->K);
    if (ws_bytes < need || !ws) return fail(NIF_ERR_WORKSPACE, "workspace too small: need %zu bytes", need);
    if (!c->d_objs) return fail(NIF_ERR_STATE, "context not prepared");
    const uint32_t* p = nullptr;
    return run_order(c, rays, ids, tmax, n, perm, ws, &p, (hipStream_t)stream, window_sorted(c),
                     reinterpret_cast<float4*>(packed));
}

extern "C" nif_status nif_query_packed(nif_ctx* c, int32_t dtype, const float* packed, const uint32_t* perm,
                                       int64_t n, float* vis, float* logits, void* stream) {
    nif_status st = check_query_args(c, dtype, packed, packed, packed, n, vis, "nif_query_packed");  // perm nullable
    if (st != NIF_OK || n == 0) return st == NIF_OK ? ok() : st;
    if (reinterpret_cast<uintptr_t>(packed) % 16 != 0)
        return fail(NIF_ERR_INVALID_ARG, "nif_query_packed: packed must be 16-byte aligned");
    if (!c->prepared[dtype]) return fail(NIF_ERR_STATE, "context not prepared for dtype %d", dtype);
    return run_query(c, dtype, nullptr, nullptr, nullptr, perm, n, vis, logits, (hipStream_t)stream, 0,
                     reinterpret_cast<const float4*>(packed));
}

extern "C" nif_status nif_query_ordered(nif_ctx* c, int32_t dtype, const float* rays, const int32_t* ids,
                                        const float* tmax, const uint32_t* perm, int64_t n, float* vis, float* logits,
                                        void* stream) {
    nif_status st = check_query_args(c, dtype, rays, ids, tmax, n, vis, "nif_query_ordered");
    if (st != NIF_OK || n == 0) return st == NIF_OK ? ok() : st;
    if (!perm) return fail(NIF_ERR_INVALID_ARG, "nif_query_ordered: NULL perm");
    if (!c->prepared[dtype]) return fail(NIF_ERR_STATE, "context not prepared for dtype %d", dtype);
    return run_query(c, dtype, rays, ids, tmax, perm, n, vis, logits, (hipStream_t)stream);
}

static void fill_common(const nif_ctx* c, FwdArgs& a) {
    a.flags = c->d_flags;
    a.use_image = c->images_ready ? c->image_mode : 0;
    for (int k = 0; k < 3 * c->d.levels; ++k) a.ioff[k] = c->ioff[k];
    a.objs = c->d_objs;
    a.num_objects = c->K;
    a.hidden = c->d.hidden_layers;
    for (int k = 0; k < 3 * c->d.levels; ++k) a.toff[k] = c->toff[k];
    for (int l = 0; l < c->d.levels; ++l) a.res[l] = c->res[l];
}

static nif_status encode_impl(nif_ctx* c, int32_t feat16, const float* rays, const int32_t* ids, const float* tmax,
                              int64_t n, void* features, int32_t* status, void* stream) {
    if (!c) return fail(NIF_ERR_INVALID_ARG, "nif_encode: NULL context");
    if (n < 0) return fail(NIF_ERR_INVALID_ARG, "nif_encode: n < 0");
    if (n == 0) return ok();
    if (!rays || !ids || !tmax || !features) return fail(NIF_ERR_INVALID_ARG, "nif_encode: NULL input or output");
    if (n > (int64_t)1 << 36) return fail(NIF_ERR_UNSUPPORTED, "nif_encode: n too large");
    if (!c->d_objs) return fail(NIF_ERR_STATE, "context not prepared");
    if (!c->images_ready && require_grids(c, "nif_encode") != NIF_OK) return NIF_ERR_STATE;  // would read grids
    FwdArgs a{};
    fill_common(c, a);
    a.rays = rays;
    a.ids = ids;
    a.tmax = tmax;
    a.n = n;
    a.features = reinterpret_cast<float*>(features);
    a.feat16 = feat16;
    a.status_out = status;
    a.pack = c->pack[kF32];
    HIP_TRY(launch_encode(c->d.levels, c->d.grid_dtype, a, c->num_cus, (hipStream_t)stream));
    return ok();
}

extern "C" nif_status nif_encode(nif_ctx* c, const float* rays, const int32_t* ids, const float* tmax, int64_t n,
                                 float* features, int32_t* status, void* stream) {
    return encode_impl(c, 0, rays, ids, tmax, n, features, status, stream);
}

extern "C" nif_status nif_encode16(nif_ctx* c, int32_t fmt, const float* rays, const int32_t* ids, const float* tmax,
                                   int64_t n, void* features, int32_t* status, void* stream) {
    if (fmt != NIF_F16 && fmt != NIF_BF16) return fail(NIF_ERR_UNSUPPORTED, "nif_encode16: format must be NIF_F16 or NIF_BF16");
    if (reinterpret_cast<uintptr_t>(features) % 8 != 0)
        return fail(NIF_ERR_INVALID_ARG, "nif_encode16: features must be 8-byte aligned");
    return encode_impl(c, fmt, rays, ids, tmax, n, features, status, stream);
}

extern "C" size_t nif_pairs_workspace_bytes(const nif_ctx* c, int64_t n_rays) {
    if (!c || n_rays < 0) return 0;
    return pairs_workspace_bytes(n_rays, c->K);
}

static nif_status expand_pairs(nif_ctx* c, const float* rays, const float* tmax, int64_t n_rays, int32_t round,
                               const uint8_t* ray_visible, int64_t max_pairs, float* pair_rays, float* pair_tmax,
                               int32_t* pair_ids, uint32_t* pair_ray, int64_t* pair_count, void* ws, size_t ws_bytes,
                               void* stream, const char* where, float* packed = nullptr, uint32_t* keys = nullptr,
                               bool grouped = false, int64_t* obj_off = nullptr) {
    if (!c) return fail(NIF_ERR_INVALID_ARG, "%s: NULL context", where);
    if (n_rays < 0 || max_pairs < 0) return fail(NIF_ERR_INVALID_ARG, "%s: negative size", where);
    if (!pair_count) return fail(NIF_ERR_INVALID_ARG, "%s: NULL pair_count", where);
    if (n_rays > 0 && (!rays || !tmax)) return fail(NIF_ERR_INVALID_ARG, "%s: NULL rays", where);
    if (max_pairs > 0 && !pair_ray) return fail(NIF_ERR_INVALID_ARG, "%s: NULL pair output", where);
    if (max_pairs > 0 && !packed && (!pair_rays || !pair_tmax || !pair_ids))
        return fail(NIF_ERR_INVALID_ARG, "%s: NULL pair output", where);
    if (packed && reinterpret_cast<uintptr_t>(packed) % 16 != 0)
        return fail(NIF_ERR_INVALID_ARG, "%s: packed must be 16-byte aligned", where);
    if (round < 0 || round > 2) return fail(NIF_ERR_INVALID_ARG, "%s: round must be 1 or 2", where);
    if (round == 2 && n_rays > 0 && !ray_visible) return fail(NIF_ERR_INVALID_ARG, "%s: NULL ray_visible", where);
    if (grouped && c->K > 64) return fail(NIF_ERR_UNSUPPORTED, "%s: at most 64 objects", where);
    if (n_rays > ((int64_t)1 << 24)) return fail(NIF_ERR_UNSUPPORTED, "%s: at most 2^24 rays per call", where);
    // per-ray counts and their scan are 32-bit: the total must stay below 2^32
    if ((uint64_t)n_rays * (uint64_t)c->K >= ((uint64_t)1 << 32))
        return fail(NIF_ERR_UNSUPPORTED, "%s: n_rays x num_objects must be below 2^32", where);
    if (!c->d_objs || !c->d_tree) return fail(NIF_ERR_STATE, "context not prepared");
    const size_t need = pairs_workspace_bytes(n_rays, c->K);
    if (ws_bytes < need || !ws) return fail(NIF_ERR_WORKSPACE, "workspace too small: need %zu bytes", need);
    HIP_TRY(launch_expand_pairs(rays, tmax, n_rays, c->tree, c->K, c->num_cus, round, ray_visible, max_pairs,
                                pair_rays, pair_tmax, pair_ids, pair_ray, pair_count, ws, (hipStream_t)stream,
                                reinterpret_cast<float4*>(packed), keys, c->d_objs,
                                order_bucket_bits(c->K, c->order_bits) == 0 && !window_sorted(c), grouped, obj_off));
    return ok();
}

extern "C" nif_status nif_expand_pairs_by_object(nif_ctx* c, const float* rays, const float* tmax, int64_t n_rays,
                                                 int64_t max_pairs, float* packed, uint32_t* pair_ray,
                                                 int64_t* pair_count, int64_t* obj_offsets, void* ws, size_t ws_bytes,
                                                 void* stream) {
    if (max_pairs > 0 && !packed) return fail(NIF_ERR_INVALID_ARG, "nif_expand_pairs_by_object: NULL packed");
    if (c && n_rays == 0 && obj_offsets) {  // no rays: every object's run is empty
        const nif_status st = expand_pairs(c, rays, tmax, 0, 0, nullptr, max_pairs, nullptr, nullptr, nullptr, pair_ray,
                                           pair_count, ws, ws_bytes, stream, "nif_expand_pairs_by_object", packed,
                                           nullptr, true, nullptr);
        if (st != NIF_OK) return st;
        HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(obj_offsets), 2 * ((int64_t)c->K + 1), 0u,
                                (hipStream_t)stream));
        return ok();
    }
    return expand_pairs(c, rays, tmax, n_rays, 0, nullptr, max_pairs, nullptr, nullptr, nullptr, pair_ray, pair_count,
                        ws, ws_bytes, stream, "nif_expand_pairs_by_object", packed, nullptr, true, obj_offsets);
}

extern "C" nif_status nif_expand_pairs_packed(nif_ctx* c, const float* rays, const float* tmax, int64_t n_rays,
                                              int64_t max_pairs, float* packed, uint32_t* pair_ray, uint32_t* keys,
                                              int64_t* pair_count, void* ws, size_t ws_bytes, void* stream) {
    if (max_pairs > 0 && !packed) return fail(NIF_ERR_INVALID_ARG, "nif_expand_pairs_packed: NULL packed");
    return expand_pairs(c, rays, tmax, n_rays, 0, nullptr, max_pairs, nullptr, nullptr, nullptr, pair_ray, pair_count,
                        ws, ws_bytes, stream, "nif_expand_pairs_packed", packed, keys);
}

extern "C" nif_status nif_expand_pairs(nif_ctx* c, const float* rays, const float* tmax, int64_t n_rays,
                                       int64_t max_pairs, float* pair_rays, float* pair_tmax, int32_t* pair_ids,
                                       uint32_t* pair_ray, int64_t* pair_count, void* ws, size_t ws_bytes,
                                       void* stream) {
    return expand_pairs(c, rays, tmax, n_rays, 0, nullptr, max_pairs, pair_rays, pair_tmax, pair_ids, pair_ray,
                        pair_count, ws, ws_bytes, stream, "nif_expand_pairs");
}

extern "C" nif_status nif_expand_pairs_round(nif_ctx* c, const float* rays, const float* tmax, int64_t n_rays,
                                             int32_t round, const uint8_t* ray_visible, int64_t max_pairs,
                                             float* pair_rays, float* pair_tmax, int32_t* pair_ids,
                                             uint32_t* pair_ray, int64_t* pair_count, void* ws, size_t ws_bytes,
                                             void* stream) {
    if (round != 1 && round != 2) return fail(NIF_ERR_INVALID_ARG, "nif_expand_pairs_round: round must be 1 or 2");
    return expand_pairs(c, rays, tmax, n_rays, round, ray_visible, max_pairs, pair_rays, pair_tmax, pair_ids,
                        pair_ray, pair_count, ws, ws_bytes, stream, "nif_expand_pairs_round");
}

static nif_status combine(nif_ctx* c, const uint32_t* pair_ray, const float* visibility, int64_t n_pairs,
                          int64_t n_rays, uint8_t* ray_visible, bool init, void* stream, const char* where) {
    if (!c) return fail(NIF_ERR_INVALID_ARG, "%s: NULL context", where);
    if (n_pairs < 0 || n_rays < 0) return fail(NIF_ERR_INVALID_ARG, "%s: negative size", where);
    if ((n_pairs > 0 && (!pair_ray || !visibility)) || (n_rays > 0 && !ray_visible))
        return fail(NIF_ERR_INVALID_ARG, "%s: NULL argument", where);
    HIP_TRY(launch_combine_pairs(pair_ray, visibility, n_pairs, n_rays, ray_visible, init, (hipStream_t)stream));
    return ok();
}

extern "C" nif_status nif_combine_pairs(nif_ctx* c, const uint32_t* pair_ray, const float* visibility, int64_t n_pairs,
                                        int64_t n_rays, uint8_t* ray_visible, void* stream) {
    return combine(c, pair_ray, visibility, n_pairs, n_rays, ray_visible, true, stream, "nif_combine_pairs");
}

extern "C" nif_status nif_combine_pairs_and(nif_ctx* c, const uint32_t* pair_ray, const float* visibility,
                                            int64_t n_pairs, int64_t n_rays, uint8_t* ray_visible, void* stream) {
    return combine(c, pair_ray, visibility, n_pairs, n_rays, ray_visible, false, stream, "nif_combine_pairs_and");
}

extern "C" nif_status nif_get_error_flags(nif_ctx* c, uint32_t* flags, int32_t clear, void* stream) {
    if (!c || !flags) return fail(NIF_ERR_INVALID_ARG, "nif_get_error_flags: NULL argument");
    *flags = 0;
    if (!c->d_flags) return ok();  // nothing has run yet
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(flags, c->d_flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (clear) HIP_TRY(launch_fill_u32(c->d_flags, 1, 0u, s));
    return ok();
}

extern "C" nif_status nif_calibrate_fp8(nif_ctx* c, int32_t mlp, const float* rays, const int32_t* ids,
                                        const float* tmax, int64_t n, float* scales, void* ws, size_t ws_bytes,
                                        void* stream) {
    if (!c) return fail(NIF_ERR_INVALID_ARG, "nif_calibrate_fp8: NULL context");
    if (mlp < 0 || mlp >= c->M) return fail(NIF_ERR_INVALID_ARG, "mlp %d out of range", mlp);
    if (n < 0) return fail(NIF_ERR_INVALID_ARG, "nif_calibrate_fp8: n < 0");
    if (n > 0 && (!rays || !ids || !tmax)) return fail(NIF_ERR_INVALID_ARG, "nif_calibrate_fp8: NULL input");
    if (n > (int64_t)1 << 31) return fail(NIF_ERR_UNSUPPORTED, "nif_calibrate_fp8: n too large");
    if (!c->masters[mlp]) return fail(NIF_ERR_STATE, "MLP %d not registered", mlp);
    if (!c->d_objs) return fail(NIF_ERR_STATE, "context not prepared");
    if (!c->images_ready && require_grids(c, "nif_calibrate_fp8") != NIF_OK) return NIF_ERR_STATE;
    const size_t need = calib_workspace_bytes(n, c->din);
    if (ws_bytes < need || !ws) return fail(NIF_ERR_WORKSPACE, "workspace too small: need %zu bytes", need);
    FwdArgs a{};
    fill_common(c, a);
    a.rays = rays;
    a.ids = ids;
    a.tmax = tmax;
    a.n = n;
    a.pack = c->pack[kF32];
    const int H = c->d.hidden_layers;
    unsigned amax[2 * kMaxHidden];
    HIP_TRY(launch_calibrate(a, c->d.levels, c->d.grid_dtype, c->num_cus, mlp, c->masters[mlp], c->din, H, ws, amax,
                             (hipStream_t)stream));
    std::vector<float> sc(2 * H);
    for (int j = 0; j < H; ++j) {
        float w, x;
        memcpy(&w, &amax[kMaxHidden + j], 4);
        memcpy(&x, &amax[j], 4);
        if (!isfinite(w) || !isfinite(x)) return fail(NIF_ERR_STATE, "non-finite weight or activation in layer %d", j + 1);
        sc[j] = w > 0.0f ? w / 448.0f : 1.0f;
        sc[H + j] = x > 0.0f ? x / 448.0f : 1.0f;
    }
    c->fp8[mlp] = sc;
    c->prepared[kFP8] = false;
    if (scales) memcpy(scales, sc.data(), sizeof(float) * 2 * H);
    return ok();
}

static nif_status mlp_impl(nif_ctx* c, int32_t dtype, int32_t feat16, int32_t mlp, const void* features, int64_t n,
                           float* logits, void* stream) {
    if (!c) return fail(NIF_ERR_INVALID_ARG, "nif_mlp: NULL context");
    if (n < 0) return fail(NIF_ERR_INVALID_ARG, "nif_mlp: n < 0");
    if (dtype < 0 || dtype > 3) return fail(NIF_ERR_UNSUPPORTED, "unknown dtype %d", dtype);
    if (mlp < 0 || mlp >= c->M) return fail(NIF_ERR_INVALID_ARG, "mlp %d out of range", mlp);
    if (n == 0) return ok();
    if (!features || !logits) return fail(NIF_ERR_INVALID_ARG, "nif_mlp: NULL input or output");
    if (n > (int64_t)1 << 36) return fail(NIF_ERR_UNSUPPORTED, "nif_mlp: n too large");
    if (!c->prepared[dtype]) return fail(NIF_ERR_STATE, "context not prepared for dtype %d", dtype);
    FwdArgs a{};
    fill_common(c, a);
    a.n = n;
    a.features = reinterpret_cast<float*>(const_cast<void*>(features));
    a.feat16 = feat16;
    a.fixed_mlp = mlp;
    a.logit = logits;
    a.vis = nullptr;
    a.packed = c->d_packed[dtype];
    a.pack = c->pack[dtype];
    a.fp8_scales = dtype == kFP8 ? c->d_scales : nullptr;
    if (feat16)
        HIP_TRY(launch_mlp16(dtype, c->d.levels, a, c->num_cus, (hipStream_t)stream));
    else
        HIP_TRY(launch_mlp(dtype, c->d.levels, a, c->num_cus, (hipStream_t)stream));
    return ok();
}

extern "C" nif_status nif_mlp(nif_ctx* c, int32_t dtype, int32_t mlp, const float* features, int64_t n,
                              float* logits, void* stream) {
    return mlp_impl(c, dtype, 0, mlp, features, n, logits, stream);
}

extern "C" nif_status nif_mlp16(nif_ctx* c, int32_t dtype, int32_t mlp, const void* features, int64_t n,
                                float* logits, void* stream) {
    if (dtype != NIF_F16 && dtype != NIF_BF16) return fail(NIF_ERR_UNSUPPORTED, "nif_mlp16: dtype must be NIF_F16 or NIF_BF16");
    if (reinterpret_cast<uintptr_t>(features) % 8 != 0)
        return fail(NIF_ERR_INVALID_ARG, "nif_mlp16: features must be 8-byte aligned");
    return mlp_impl(c, dtype, dtype, mlp, features, n, logits, stream);
}

extern "C" size_t nif_touched_bytes(const nif_ctx* c) {
    if (!c) return 0;
    const int64_t chunks = (c->grid_elems + 63) / 64;  // one flag byte per 64 latents
    return (size_t)((chunks + 3) / 4) * 4;
}

extern "C" nif_status nif_set_object_train(nif_ctx* c, int32_t obj, float* grad, float* m, float* v,
                                           void* touched) {
    if (!c || !grad || !m || !v || !touched) return fail(NIF_ERR_INVALID_ARG, "nif_set_object_train: NULL argument");
    if (obj < 0 || obj >= c->K) return fail(NIF_ERR_INVALID_ARG, "object %d out of range", obj);
    ObjHost& o = c->objs[obj];
    o.grad = grad;
    o.m = m;
    o.v = v;
    o.touched = touched;
    c->train_tab_dirty = true;
    return ok();
}

extern "C" nif_status nif_set_mlp_train(nif_ctx* c, int32_t mlp, float* m, float* v) {
    if (!c || !m || !v) return fail(NIF_ERR_INVALID_ARG, "nif_set_mlp_train: NULL argument");
    if (mlp < 0 || mlp >= c->M) return fail(NIF_ERR_INVALID_ARG, "mlp %d out of range", mlp);
    c->mlp_m[mlp] = m;
    c->mlp_v[mlp] = v;
    return ok();
}

static size_t train_bytes(const nif_ctx* c, int64_t n) {
    return train_workspace_bytes(n, c->din, c->d.hidden_layers, c->P, nullptr) +
           (uses_order(c, n) ? order_workspace_bytes(n, c->K) : 0);
}

// Training step (labels, optional Adam) or backward pass of a given upstream
// gradient (grad_y; gradients only).
static nif_status train_common(nif_ctx* c, int32_t mlp, const float* rays, const int32_t* ids, const float* tmax,
                               const uint8_t* labels, const float* grad_y, int64_t n, int32_t step,
                               const nif_adam* adam, float* loss, float* mlp_grad, void* ws, size_t ws_bytes,
                               void* stream, const float* t_hit = nullptr) {
    nif_status st = NIF_OK;
    if (mlp < 0 || mlp >= c->M) return fail(NIF_ERR_INVALID_ARG, "mlp %d out of range", mlp);
    if (adam && step < 1) return fail(NIF_ERR_INVALID_ARG, "step must be >= 1");
    if (adam && !(adam->lr > 0.0f && adam->beta1 >= 0.0f && adam->beta1 < 1.0f && adam->beta2 >= 0.0f &&
                  adam->beta2 < 1.0f && adam->eps >= 0.0f))
        return fail(NIF_ERR_INVALID_ARG, "invalid Adam hyper-parameters");
    if (n == 0) return ok();
    if (!c->d_objs) return fail(NIF_ERR_STATE, "context not prepared");
    if (require_grids(c, "training") != NIF_OK) return NIF_ERR_STATE;
    if (!c->masters[mlp]) return fail(NIF_ERR_STATE, "MLP %d not registered", mlp);
    if (adam && (!c->mlp_m[mlp] || !c->mlp_v[mlp])) return fail(NIF_ERR_STATE, "MLP %d has no Adam moments", mlp);
    std::vector<int32_t> objs;
    for (int k = 0; k < c->K; ++k)
        if (c->objs[k].mlp == mlp) {
            const ObjHost& o = c->objs[k];
            if (!o.grad || !o.touched || (adam && (!o.m || !o.v)))
                return fail(NIF_ERR_STATE, "object %d has no training buffers", k);
            objs.push_back(k);
        }
    const size_t need = train_bytes(c, n);
    if (ws_bytes < need || !ws) return fail(NIF_ERR_WORKSPACE, "workspace too small: need %zu bytes", need);
    hipStream_t s = (hipStream_t)stream;
    const int K = c->K;
    if (!c->d_train_tab) HIP_TRY(hipMalloc(&c->d_train_tab, sizeof(void*) * 5 * K));
    if (c->train_tab_dirty) {
        std::vector<void*> tab((size_t)5 * K, nullptr);
        for (int k = 0; k < K; ++k) {
            tab[0 * K + k] = c->objs[k].grad;
            tab[1 * K + k] = c->objs[k].m;
            tab[2 * K + k] = c->objs[k].v;
            tab[3 * K + k] = c->objs[k].touched;
            tab[4 * K + k] = c->objs[k].grid;
        }
        HIP_TRY(hipStreamSynchronize(s));
        HIP_TRY(hipMemcpy(c->d_train_tab, tab.data(), sizeof(void*) * tab.size(), hipMemcpyHostToDevice));
        c->train_tab_dirty = false;
    }
    const PackInfo& P32 = c->pack[kF32];
    if (!c->d_train_fwd) HIP_TRY(hipMalloc(&c->d_train_fwd, P32.bytes));
    if (!c->d_train_bwd) HIP_TRY(hipMalloc(&c->d_train_bwd, backward_image_bytes(c->d.hidden_layers)));
    HIP_TRY(launch_pack_forward(c->masters[mlp], c->d_train_fwd, P32, kF32, c->din, c->d.width, nullptr, s));
    HIP_TRY(launch_pack_backward(c->masters[mlp], c->d_train_bwd, c->d.hidden_layers, c->din, c->d.width, s));
    TrainArgs A{};
    uint8_t* wsp = reinterpret_cast<uint8_t*>(ws);
    const size_t tb = train_workspace_bytes(n, c->din, c->d.hidden_layers, c->P, nullptr);
    if (uses_order(c, n)) {
        st = run_order(c, rays, ids, tmax, n, nullptr, wsp + tb, &A.perm, s);
        if (st != NIF_OK) return st;
    }
    A.rays = rays;
    A.ids = ids;
    A.tmax = tmax;
    A.labels = labels;
    A.grad_y = grad_y;
    A.t_hit = t_hit;
    A.n = n;
    A.objs = c->d_objs;
    A.num_objects = K;
    A.mlp = mlp;
    A.hidden = c->d.hidden_layers;
    A.din = c->din;
    A.P = c->P;
    for (int k = 0; k < 3 * c->d.levels; ++k) A.toff[k] = c->toff[k];
    for (int l = 0; l < c->d.levels; ++l) A.res[l] = c->res[l];
    A.fwd = reinterpret_cast<const float*>(c->d_train_fwd);
    A.pack = P32;
    A.bwd = c->d_train_bwd;
    A.grid_grad = reinterpret_cast<float* const*>(c->d_train_tab + 0 * K);
    A.grid_m = reinterpret_cast<float* const*>(c->d_train_tab + 1 * K);
    A.grid_v = reinterpret_cast<float* const*>(c->d_train_tab + 2 * K);
    A.touched = reinterpret_cast<uint8_t* const*>(c->d_train_tab + 3 * K);
    A.grids = c->d_train_tab + 4 * K;
    A.master = c->masters[mlp];
    A.mlp_m = c->mlp_m[mlp];
    A.mlp_v = c->mlp_v[mlp];
    A.loss_out = loss;
    A.grad_out = mlp_grad;
    A.apply_adam = adam ? 1 : 0;
    if (adam) {
        A.adam.lr = adam->lr;
        A.adam.beta1 = adam->beta1;
        A.adam.beta2 = adam->beta2;
        A.adam.eps = adam->eps;
        A.adam.bc1 = (float)(1.0 - pow((double)adam->beta1, step));
        A.adam.bc2 = (float)(1.0 - pow((double)adam->beta2, step));
    }
    std::vector<int64_t> elems(K, c->grid_elems);
    HIP_TRY(launch_train(A, wsp, objs.data(), (int32_t)objs.size(), elems.data(), c->d.grid_dtype, c->d.levels,
                         c->num_cus, s));
    if (adam) invalidate(c);  // the masters changed: packed copies are stale
    return ok();
}

extern "C" nif_status nif_train_step(nif_ctx* c, int32_t mlp, const float* rays, const int32_t* ids,
                                     const float* tmax, const uint8_t* labels, int64_t n, int32_t step,
                                     const nif_adam* adam, float* loss, float* mlp_grad, void* ws, size_t ws_bytes,
                                     void* stream) {
    nif_status st = check_query_args(c, 0, rays, ids, tmax, n, labels, "nif_train_step");
    if (st != NIF_OK) return st;
    return train_common(c, mlp, rays, ids, tmax, labels, nullptr, n, step, adam, loss, mlp_grad, ws, ws_bytes,
                        stream);
}

extern "C" nif_status nif_train_step_depth(nif_ctx* c, int32_t mlp, const float* rays, const int32_t* ids,
                                           const float* tmax, const float* t_hit, int64_t n, int32_t step,
                                           const nif_adam* adam, float* loss, float* mlp_grad, void* ws,
                                           size_t ws_bytes, void* stream) {
    nif_status st = check_query_args(c, 0, rays, ids, tmax, n, t_hit, "nif_train_step_depth");
    if (st != NIF_OK) return st;
    return train_common(c, mlp, rays, ids, tmax, nullptr, nullptr, n, step, adam, loss, mlp_grad, ws, ws_bytes,
                        stream, t_hit);
}

extern "C" nif_status nif_depth_from_visibility(nif_ctx* c, const float* rays, const int32_t* ids, const float* tmax,
                                                const float* visibility, int64_t n, float* depth, void* stream) {
    nif_status st = check_query_args(c, 0, rays, ids, tmax, n, visibility, "nif_depth_from_visibility");
    if (st != NIF_OK || n == 0) return st == NIF_OK ? ok() : st;
    if (!depth) return fail(NIF_ERR_INVALID_ARG, "nif_depth_from_visibility: NULL depth");
    if (!c->d_objs) return fail(NIF_ERR_STATE, "context not prepared");
    HIP_TRY(launch_depth_from_visibility(rays, ids, tmax, visibility, n, c->d_objs, c->K, depth, c->num_cus,
                                         (hipStream_t)stream));
    return ok();
}

extern "C" nif_status nif_backward(nif_ctx* c, int32_t mlp, const float* rays, const int32_t* ids,
                                   const float* tmax, const float* grad_visibility, int64_t n, float* mlp_grad,
                                   void* ws, size_t ws_bytes, void* stream) {
    nif_status st = check_query_args(c, 0, rays, ids, tmax, n, grad_visibility, "nif_backward");
    if (st != NIF_OK) return st;
    return train_common(c, mlp, rays, ids, tmax, nullptr, grad_visibility, n, 1, nullptr, nullptr, mlp_grad, ws,
                        ws_bytes, stream);
}

// ---------------------------------------------------------------------------
// Query plans: one schedule (ordering variant + persistent grid size) chosen by
// timing the candidates on the caller's buffers, then captured into a HIP
// graph that replays the ordering kernels and the fused query kernel.
// ---------------------------------------------------------------------------
struct Sched {
    int32_t order;          // 0 none, 1 bucket order, 2 bucket order + window sort, 3 by object alone
    int32_t blocks_per_cu;  // persistent grid: blocks per compute unit
    int32_t shape;          // tile shape of the fused kernel: gathers issued together, waves per SIMD
};

// The tile shape's parameters as the fused kernel instantiates them (8-level
// binary16 grids; other grids run shape 0): gathers issued together per lane
// half (image / grid path) and the waves per SIMD the registers are cut for.
static void shape_params(int32_t shape, int32_t dtype, int32_t levels, int32_t image, int32_t* batch, int32_t* wpe) {
    const int NL = 3 * levels / 2;
    *batch = shape == 1 ? (image ? NL : NL / 2) : shape == 2 ? 3 : (image ? 6 : NL);
    *wpe = shape == 1 ? 2 : shape == 2 ? 4 : (dtype == NIF_F32 ? 2 : 3);
}

struct nif_plan {
    nif_ctx* c = nullptr;
    int32_t dtype = 0;
    const float* rays = nullptr;
    const int32_t* ids = nullptr;
    const float* tmax = nullptr;
    int64_t n = 0;
    float* vis = nullptr;
    float* logits = nullptr;
    void* ws = nullptr;
    Sched sched{2, 8, 0};
    float tuned_us = -1.0f;  // time of the chosen schedule (-1: given, not tuned)
    int32_t candidates = 0;
    bool from_cache = false;
    uint64_t epoch = 0;  // the context's epoch at capture
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

static nif_status plan_run(nif_plan* p, const Sched& sc, hipStream_t s) {
    const uint32_t* perm = nullptr;
    float4* qrec = nullptr;
    uint32_t* ctr = tile_ctr_in(p->c, p->ws, p->n);
    if (sc.order > 0) {  // plans order by their own schedule, not by the context's NIF_OPT_ORDER_BITS
        qrec = records_in(p->c, p->ws, p->n);
        nif_status st = run_order(p->c, p->rays, p->ids, p->tmax, p->n, nullptr, p->ws, &perm, s, sc.order == 2, qrec,
                                  ctr, sc.order == 3 ? 0 : -1);
        if (st != NIF_OK) return st;
    }
    return run_query(p->c, p->dtype, p->rays, p->ids, p->tmax, perm, p->n, p->vis, p->logits, s, sc.blocks_per_cu,
                     qrec, sc.shape, ctr, sc.order > 0);
}

// Tuning cache: a text file of one JSON object per line, {"key": "...",
// "order": o, "blocks_per_cu": b, "shape": s}, named by the environment
// variable NIF_PLAN_CACHE (no cache when unset).  The key holds the device
// architecture and compute-unit count, the model shape, the number of objects
// and MLPs, the query image mode, the dtype and n rounded up to a power of two.
static std::string plan_key(const nif_ctx* c, int32_t dtype, int64_t n) {
    hipDeviceProp_t prop{};
    const char* arch = hipGetDeviceProperties(&prop, c->device) == hipSuccess ? prop.gcnArchName : "unknown";
    int64_t nb = 1;
    while (nb < n) nb <<= 1;
    char buf[512];
    snprintf(buf, sizeof buf, "%s|cu%d|L%d r%d-%d F%d g%d H%d W%d|K%d M%d|img%d|dtype%d|n%lld", arch, c->num_cus,
             c->d.levels, c->d.res_min, c->d.res_max, c->d.feats, c->d.grid_dtype, c->d.hidden_layers, c->d.width, c->K,
             c->M, c->image_mode, dtype, (long long)nb);
    return buf;
}

static bool parse_int_key(const char* js, const char* key, int32_t* v);

static bool cache_lookup(const std::string& key, Sched* sc) {
    const char* path = getenv("NIF_PLAN_CACHE");
    if (!path || !*path) return false;
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char line[1024];
    const std::string want = "\"key\": \"" + key + "\"";
    bool found = false;
    while (fgets(line, sizeof line, f)) {
        if (!strstr(line, want.c_str())) continue;
        Sched s{2, 8, 0};
        if (parse_int_key(line, "\"order\"", &s.order) && parse_int_key(line, "\"blocks_per_cu\"", &s.blocks_per_cu) &&
            parse_int_key(line, "\"shape\"", &s.shape) && s.order >= 0 && s.order <= 3 && s.blocks_per_cu >= 1 &&
            s.blocks_per_cu <= 32 && s.shape >= 0 && s.shape <= 2) {
            *sc = s;  // the last matching line wins
            found = true;
        }
    }
    fclose(f);
    return found;
}

static void cache_store(const std::string& key, const Sched& sc, float us) {
    const char* path = getenv("NIF_PLAN_CACHE");
    if (!path || !*path) return;
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "{\"key\": \"%s\", \"order\": %d, \"blocks_per_cu\": %d, \"shape\": %d, \"tuned_us\": %.3f}\n",
            key.c_str(), sc.order, sc.blocks_per_cu, sc.shape, (double)us);
    fclose(f);
}

static bool parse_int_key(const char* js, const char* key, int32_t* v) {
    const char* q = strstr(js, key);
    if (!q) return false;
    q = strchr(q + strlen(key), ':');
    if (!q) return false;
    char* end = nullptr;
    const long x = strtol(q + 1, &end, 10);
    if (end == q + 1) return false;
    *v = (int32_t)x;
    return true;
}

extern "C" size_t nif_plan_workspace_bytes(const nif_ctx* c, int64_t n) {
    if (!c || n <= 0) return 0;
    return order_packed_bytes(c, n);
}

extern "C" nif_status nif_plan_create(nif_ctx* c, int32_t dtype, const float* rays, const int32_t* ids,
                                      const float* tmax, int64_t n, float* vis, float* logits, void* ws,
                                      size_t ws_bytes, const char* tuning, void* stream, nif_plan** out) {
    if (!out) return fail(NIF_ERR_INVALID_ARG, "nif_plan_create: NULL out");
    *out = nullptr;
    nif_status st = check_query_args(c, dtype, rays, ids, tmax, n, vis, "nif_plan_create");
    if (st != NIF_OK) return st;
    if (n == 0) return fail(NIF_ERR_INVALID_ARG, "nif_plan_create: n must be > 0");
    if (!c->prepared[dtype]) return fail(NIF_ERR_STATE, "context not prepared for dtype %d", dtype);
    const size_t need = order_packed_bytes(c, n);
    if (ws_bytes < need || !ws) return fail(NIF_ERR_WORKSPACE, "workspace too small: need %zu bytes", need);
    std::unique_ptr<nif_plan> p(new nif_plan);
    p->c = c;
    p->dtype = dtype;
    p->rays = rays;
    p->ids = ids;
    p->tmax = tmax;
    p->n = n;
    p->vis = vis;
    p->logits = logits;
    p->ws = ws;
    hipStream_t s = (hipStream_t)stream;
    const std::string key = plan_key(c, dtype, n);
    Sched cached{2, 8, 0};
    if (tuning) {
        Sched sc{2, 8, 0};
        if (!parse_int_key(tuning, "\"order\"", &sc.order) || !parse_int_key(tuning, "\"blocks_per_cu\"", &sc.blocks_per_cu))
            return fail(NIF_ERR_INVALID_ARG, "tuning string lacks \"order\" or \"blocks_per_cu\"");
        (void)parse_int_key(tuning, "\"shape\"", &sc.shape);  // optional, default 0
        if (sc.order < 0 || sc.order > 3 || sc.blocks_per_cu < 1 || sc.blocks_per_cu > 32 || sc.shape < 0 ||
            sc.shape > 2)
            return fail(NIF_ERR_INVALID_ARG, "tuning out of range (order 0..3, blocks_per_cu 1..32, shape 0..2)");
        p->sched = sc;
    } else if (cache_lookup(key, &cached)) {
        p->sched = cached;
        p->from_cache = true;
    } else {
        // autotune: every candidate once untimed, then the best of three timed runs.
        // Orderings x persistent grid sizes x tile shapes (shapes only where the
        // kernel has them: 8-level binary16 grids)
        std::vector<Sched> cand;
        const int nshape = c->d.levels == 8 && c->d.grid_dtype == NIF_F16 ? 3 : 1;
        for (int o = 0; o <= 3; ++o)
            for (int b : {4, 8, 16, 32})
                for (int sh = 0; sh < nshape; ++sh)
                    if (!(o == 0 && b == 4)) cand.push_back(Sched{o, b, sh});
        hipEvent_t e0, e1;
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        float best = -1.0f;
        for (const Sched& sc : cand) {
            st = plan_run(p.get(), sc, s);
            float tmin = 1e30f;
            for (int r = 0; r < 3 && st == NIF_OK; ++r) {
                (void)hipEventRecord(e0, s);
                st = plan_run(p.get(), sc, s);
                (void)hipEventRecord(e1, s);
                if (hipEventSynchronize(e1) != hipSuccess) st = fail(NIF_ERR_HIP, "event synchronisation failed");
                float ms = 0.0f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                tmin = ms < tmin ? ms : tmin;
            }
            if (st != NIF_OK) break;
            ++p->candidates;
            if (best < 0.0f || tmin < best) {
                best = tmin;
                p->sched = sc;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (st != NIF_OK) return st;
        p->tuned_us = best * 1e3f;
        cache_store(key, p->sched, p->tuned_us);
    }
    // capture on a private stream (the caller's may be the legacy default stream)
    hipStream_t cs;
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
        st = plan_run(p.get(), p->sched, cs);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(cs, &g);
        p->graph = g;
        if (e == hipSuccess && st == NIF_OK) e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
    }
    (void)hipStreamDestroy(cs);
    if (st != NIF_OK) {
        if (p->graph) (void)hipGraphDestroy(p->graph);
        return st;
    }
    if (e != hipSuccess) {
        if (p->graph) (void)hipGraphDestroy(p->graph);
        return fail(NIF_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
    }
    p->epoch = c->epoch;
    *out = p.release();
    return ok();
}

extern "C" nif_status nif_plan_launch(nif_plan* p, void* stream) {
    if (!p || !p->exec) return fail(NIF_ERR_INVALID_ARG, "nif_plan_launch: NULL plan");
    if (p->c->epoch != p->epoch)
        return fail(NIF_ERR_STATE, "nif_plan_launch: the context changed since capture (object, image or option); "
                                   "create a new plan");
    if (!p->c->prepared[p->dtype])
        return fail(NIF_ERR_STATE, "nif_plan_launch: context not prepared for dtype %d (weights changed since the "
                                   "last nif_prepare)", p->dtype);
    HIP_TRY(hipGraphLaunch(p->exec, (hipStream_t)stream));
    return ok();
}

extern "C" nif_status nif_plan_tuning(const nif_plan* p, char* buf, size_t buf_bytes) {
    if (!p || !buf) return fail(NIF_ERR_INVALID_ARG, "nif_plan_tuning: NULL argument");
    int32_t batch = 0, wpe = 0;
    shape_params(p->sched.shape, p->dtype, p->c->d.levels, p->c->images_ready ? p->c->image_mode : 0, &batch, &wpe);
    const int k = snprintf(buf, buf_bytes,
                           "{\"order\": %d, \"blocks_per_cu\": %d, \"shape\": %d, \"gather_batch\": %d, "
                           "\"waves_per_simd\": %d, \"queries_per_wave\": %d, \"waves_per_block\": %d, "
                           "\"tuned_us\": %.3f, \"candidates\": %d, \"from_cache\": %s}",
                           p->sched.order, p->sched.blocks_per_cu, p->sched.shape, batch, wpe, kQueriesPerWave,
                           kBlock / 64, (double)p->tuned_us, p->candidates, p->from_cache ? "true" : "false");
    if (k < 0 || (size_t)k >= buf_bytes) return fail(NIF_ERR_INVALID_ARG, "nif_plan_tuning: buffer too small");
    return ok();
}

extern "C" void nif_plan_destroy(nif_plan* p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    delete p;
}

// ---------------------------------------------------------------------------
// The paper's own networks (Sec. 3.1, Sec. 3.2, Sec. 5, Table 1): per object a
// binary16 grid buffer for each network, one MLP per network shared by all
// objects.  The MLPs are padded on the host to the 64-wide MFMA tiling (zero
// rows and columns add exact zeros) and, for the inner network, the 13 inputs
// are placed as [position 5, distance 0-1 | direction 5, distance 2, 0] so
// that each half of a query's lanes holds one grid's latents.
// ---------------------------------------------------------------------------
struct PaperNet {
    int din, din_pad, width, hidden;
};
static const PaperNet kPaperNets[2] = {{6, 6, 64, 2}, {13, 14, 48, 3}};

static int64_t paper_params(int net) {
    const PaperNet& p = kPaperNets[net];
    return (int64_t)p.width * p.din + (int64_t)(p.hidden - 1) * p.width * p.width + p.width;
}

static int64_t paper_grid_elems(int net) { return net == 0 ? 2LL * 256 * 256 * 3 : 2LL * 128 * 128 * 5 + 128 * 3; }

// padded input column -> original column of W1 (-1: zero)
static int paper_w1_column(int net, int c) {
    if (net == 0) return c;
    static const int map[14] = {0, 1, 2, 3, 4, 10, 11, 5, 6, 7, 8, 9, 12, -1};
    return map[c];
}

struct nif_paper {
    int32_t K = 0;
    int num_cus = 256;
    std::vector<PaperObj> objs;
    std::vector<bool> set;
    float* d_master[2] = {nullptr, nullptr};
    uint8_t* d_packed[2][3] = {};
    PackInfo pack[2][3] = {};
    bool prepared[3] = {false, false, false};
    PaperObj* d_objs = nullptr;
    // training: per network the caller's master and moments, per object and
    // network the latent gradient and moments; device tables of those pointers
    float* w[2] = {nullptr, nullptr};
    float* mlp_m[2] = {nullptr, nullptr};
    float* mlp_v[2] = {nullptr, nullptr};
    std::vector<float*> gg[2], gm[2], gv[2];
    void** d_tab[2] = {nullptr, nullptr};
    bool tab_dirty[2] = {true, true};
};

extern "C" int64_t nif_paper_mlp_params(int32_t network) {
    return network == 0 || network == 1 ? paper_params(network) : -1;
}

extern "C" int64_t nif_paper_grid_elems(int32_t network) {
    return network == 0 || network == 1 ? paper_grid_elems(network) : -1;
}

extern "C" nif_status nif_paper_create(int32_t num_objects, nif_paper** out) {
    if (!out) return fail(NIF_ERR_INVALID_ARG, "nif_paper_create: NULL out");
    *out = nullptr;
    if (num_objects < 1) return fail(NIF_ERR_INVALID_ARG, "nif_paper_create: need >= 1 object");
    nif_paper* p = new nif_paper;
    p->K = num_objects;
    p->objs.resize(num_objects);
    p->set.assign(num_objects, false);
    for (int n = 0; n < 2; ++n) {
        p->gg[n].assign(num_objects, nullptr);
        p->gm[n].assign(num_objects, nullptr);
        p->gv[n].assign(num_objects, nullptr);
    }
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
        p->num_cus = cus;
    *out = p;
    return ok();
}

extern "C" void nif_paper_destroy(nif_paper* p) {
    if (!p) return;
    for (int n = 0; n < 2; ++n) {
        if (p->d_master[n]) (void)hipFree(p->d_master[n]);
        for (int f = 0; f < 3; ++f)
            if (p->d_packed[n][f]) (void)hipFree(p->d_packed[n][f]);
    }
    if (p->d_objs) (void)hipFree(p->d_objs);
    for (int n = 0; n < 2; ++n)
        if (p->d_tab[n]) (void)hipFree(p->d_tab[n]);
    delete p;
}

extern "C" nif_status nif_paper_set_object(nif_paper* p, int32_t obj, const float* aabb, void* outer_grid,
                                           void* inner_grid) {
    if (!p || !aabb || !outer_grid || !inner_grid) return fail(NIF_ERR_INVALID_ARG, "nif_paper_set_object: NULL argument");
    if (obj < 0 || obj >= p->K) return fail(NIF_ERR_INVALID_ARG, "object %d out of range", obj);
    for (int a = 0; a < 3; ++a)
        if (!(isfinite(aabb[a]) && isfinite(aabb[3 + a]) && aabb[3 + a] > aabb[a]))
            return fail(NIF_ERR_INVALID_ARG, "object %d: AABB must be finite with hi > lo on every axis", obj);
    PaperObj& o = p->objs[obj];
    for (int a = 0; a < 3; ++a) {
        o.lo[a] = aabb[a];
        o.hi[a] = aabb[3 + a];
        o.c[a] = (float)(0.5 * ((double)aabb[a] + (double)aabb[3 + a]));
        o.ih[a] = (float)(2.0 / ((double)aabb[3 + a] - (double)aabb[a]));
    }
    o.grid[0] = outer_grid;
    o.grid[1] = inner_grid;
    p->set[obj] = true;
    for (bool& b : p->prepared) b = false;
    p->tab_dirty[0] = p->tab_dirty[1] = true;
    return ok();
}

extern "C" nif_status nif_paper_init_grid(nif_paper* p, int32_t obj, int32_t network, uint64_t seed, float amp,
                                          void* stream) {
    if (!p) return fail(NIF_ERR_INVALID_ARG, "nif_paper_init_grid: NULL handle");
    if (obj < 0 || obj >= p->K || !p->set[obj]) return fail(NIF_ERR_INVALID_ARG, "object %d not registered", obj);
    if (network != 0 && network != 1) return fail(NIF_ERR_INVALID_ARG, "network must be 0 (outer) or 1 (inner)");
    if (!isfinite(amp) || amp < 0.0f) return fail(NIF_ERR_INVALID_ARG, "amp must be finite and >= 0");
    HIP_TRY(launch_init_grid(const_cast<void*>(p->objs[obj].grid[network]), NIF_F16, paper_grid_elems(network), seed,
                             2ull * (uint64_t)obj + (uint64_t)network, amp, (hipStream_t)stream));
    return ok();
}

extern "C" nif_status nif_paper_set_mlp(nif_paper* p, int32_t network, const float* w, void* stream) {
    if (!p || !w) return fail(NIF_ERR_INVALID_ARG, "nif_paper_set_mlp: NULL argument");
    if (network != 0 && network != 1) return fail(NIF_ERR_INVALID_ARG, "network must be 0 (outer) or 1 (inner)");
    const PaperNet& N = kPaperNets[network];
    const int64_t P = paper_params(network);
    std::vector<float> src((size_t)P);
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(src.data(), w, sizeof(float) * P, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    // padded binary32 master: W1 [64][din_pad], W2..WH [64][64], w_out [64]
    const int64_t Pp = (int64_t)kWidth * N.din_pad + (int64_t)(N.hidden - 1) * kWidth * kWidth + kWidth;
    std::vector<float> dst((size_t)Pp, 0.0f);
    for (int r = 0; r < N.width; ++r)
        for (int c = 0; c < N.din_pad; ++c) {
            const int oc = paper_w1_column(network, c);
            if (oc >= 0) dst[(size_t)r * N.din_pad + c] = src[(size_t)r * N.din + oc];
        }
    int64_t so = (int64_t)N.width * N.din, dp = (int64_t)kWidth * N.din_pad;
    for (int j = 1; j < N.hidden; ++j) {
        for (int r = 0; r < N.width; ++r)
            for (int c = 0; c < N.width; ++c) dst[(size_t)(dp + (int64_t)r * kWidth + c)] = src[(size_t)(so + (int64_t)r * N.width + c)];
        so += (int64_t)N.width * N.width;
        dp += (int64_t)kWidth * kWidth;
    }
    for (int c = 0; c < N.width; ++c) dst[(size_t)(dp + c)] = src[(size_t)(so + c)];
    if (!p->d_master[network]) HIP_TRY(hipMalloc(&p->d_master[network], sizeof(float) * Pp));
    HIP_TRY(hipMemcpy(p->d_master[network], dst.data(), sizeof(float) * Pp, hipMemcpyHostToDevice));
    for (bool& b : p->prepared) b = false;
    return ok();
}

extern "C" nif_status nif_paper_prepare(nif_paper* p, int32_t dtype, void* stream) {
    if (!p) return fail(NIF_ERR_INVALID_ARG, "nif_paper_prepare: NULL handle");
    if (dtype < 0 || dtype > 2) return fail(NIF_ERR_UNSUPPORTED, "the paper's networks run in binary32, FP16 or BF16");
    for (int k = 0; k < p->K; ++k)
        if (!p->set[k]) return fail(NIF_ERR_STATE, "object %d not registered", k);
    for (int n = 0; n < 2; ++n)
        if (!p->d_master[n]) return fail(NIF_ERR_STATE, "%s network has no weights", n ? "inner" : "outer");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipStreamSynchronize(s));
    if (!p->d_objs) HIP_TRY(hipMalloc(&p->d_objs, sizeof(PaperObj) * p->K));
    HIP_TRY(hipMemcpy(p->d_objs, p->objs.data(), sizeof(PaperObj) * p->K, hipMemcpyHostToDevice));
    for (int n = 0; n < 2; ++n) {
        const PaperNet& N = kPaperNets[n];
        PackInfo P = pack_info(dtype, N.din_pad, N.hidden);
        if (!p->d_packed[n][dtype]) HIP_TRY(hipMalloc(&p->d_packed[n][dtype], (size_t)P.bytes));
        p->pack[n][dtype] = P;
        HIP_TRY(launch_pack_forward(p->d_master[n], p->d_packed[n][dtype], P, dtype, N.din_pad, kWidth, nullptr, s));
    }
    p->prepared[dtype] = true;
    return ok();
}

extern "C" nif_status nif_paper_query(nif_paper* p, int32_t dtype, const float* rays, const int32_t* ids,
                                      const float* tmax, int64_t n, float* vis, float* logits, void* stream) {
    if (!p) return fail(NIF_ERR_INVALID_ARG, "nif_paper_query: NULL handle");
    if (n < 0) return fail(NIF_ERR_INVALID_ARG, "nif_paper_query: n < 0");
    if (dtype < 0 || dtype > 2) return fail(NIF_ERR_UNSUPPORTED, "the paper's networks run in binary32, FP16 or BF16");
    if (n == 0) return ok();
    if (!rays || !ids || !tmax || !vis) return fail(NIF_ERR_INVALID_ARG, "nif_paper_query: NULL input or output");
    if (n > ((int64_t)1 << 31) - 1) return fail(NIF_ERR_UNSUPPORTED, "nif_paper_query: n must be below 2^31");
    if (!p->prepared[dtype]) return fail(NIF_ERR_STATE, "not prepared for dtype %d", dtype);
    PaperArgs a{};
    a.rays = rays;
    a.ids = ids;
    a.tmax = tmax;
    a.n = n;
    a.vis = vis;
    a.logit = logits;
    a.objs = p->d_objs;
    a.num_objects = p->K;
    for (int net = 0; net < 2; ++net) {
        a.hidden[net] = kPaperNets[net].hidden;
        a.packed[net] = p->d_packed[net][dtype];
        a.pack[net] = p->pack[net][dtype];
    }
    HIP_TRY(launch_paper(dtype, a, p->num_cus, (hipStream_t)stream));
    return ok();
}

extern "C" nif_status nif_paper_set_train(nif_paper* p, int32_t network, float* w, float* m, float* v, void* stream) {
    if (!p || !w || !m || !v) return fail(NIF_ERR_INVALID_ARG, "nif_paper_set_train: NULL argument");
    if (network != 0 && network != 1) return fail(NIF_ERR_INVALID_ARG, "network must be 0 (outer) or 1 (inner)");
    nif_status st = nif_paper_set_mlp(p, network, w, stream);  // the inference master starts from w
    if (st != NIF_OK) return st;
    p->w[network] = w;
    p->mlp_m[network] = m;
    p->mlp_v[network] = v;
    return ok();
}

extern "C" nif_status nif_paper_set_object_train(nif_paper* p, int32_t obj, int32_t network, float* grid_grad,
                                                 float* grid_m, float* grid_v) {
    if (!p || !grid_grad || !grid_m || !grid_v) return fail(NIF_ERR_INVALID_ARG, "nif_paper_set_object_train: NULL argument");
    if (obj < 0 || obj >= p->K || !p->set[obj]) return fail(NIF_ERR_INVALID_ARG, "object %d not registered", obj);
    if (network != 0 && network != 1) return fail(NIF_ERR_INVALID_ARG, "network must be 0 (outer) or 1 (inner)");
    p->gg[network][obj] = grid_grad;
    p->gm[network][obj] = grid_m;
    p->gv[network][obj] = grid_v;
    p->tab_dirty[network] = true;
    return ok();
}

extern "C" size_t nif_paper_train_workspace_bytes(const nif_paper* p, int32_t network, int64_t n) {
    if (!p || n < 0 || (network != 0 && network != 1)) return 0;
    return paper_train_workspace_bytes(network, n);
}

static nif_status paper_train_common(nif_paper* p, int32_t network, const float* rays, const int32_t* ids,
                                     const float* tmax, const uint8_t* labels, const float* grad_y, int64_t n,
                                     int32_t step, const nif_adam* adam, float* loss, float* mlp_grad, void* ws,
                                     size_t ws_bytes, void* stream) {
    if (!p) return fail(NIF_ERR_INVALID_ARG, "nif_paper_train_step: NULL handle");
    if (network != 0 && network != 1) return fail(NIF_ERR_INVALID_ARG, "network must be 0 (outer) or 1 (inner)");
    if (n < 0) return fail(NIF_ERR_INVALID_ARG, "nif_paper_train_step: n < 0");
    if (n > 0 && (!rays || !ids || !tmax || (!labels && !grad_y)))
        return fail(NIF_ERR_INVALID_ARG, "nif_paper_train_step: NULL input");
    if (n > ((int64_t)1 << 31) - 1) return fail(NIF_ERR_UNSUPPORTED, "nif_paper_train_step: n must be below 2^31");
    if (adam && step < 1) return fail(NIF_ERR_INVALID_ARG, "step must be >= 1");
    if (adam && !(adam->lr > 0.0f && adam->beta1 >= 0.0f && adam->beta1 < 1.0f && adam->beta2 >= 0.0f &&
                  adam->beta2 < 1.0f && adam->eps >= 0.0f))
        return fail(NIF_ERR_INVALID_ARG, "invalid Adam hyper-parameters");
    if (!p->w[network]) return fail(NIF_ERR_STATE, "network %d has no training buffers", network);
    for (int k = 0; k < p->K; ++k) {
        if (!p->set[k]) return fail(NIF_ERR_STATE, "object %d not registered", k);
        if (!p->gg[network][k]) return fail(NIF_ERR_STATE, "object %d has no training buffers for network %d", k, network);
    }
    const size_t need = paper_train_workspace_bytes(network, n);
    if (ws_bytes < need || !ws) return fail(NIF_ERR_WORKSPACE, "workspace too small: need %zu bytes", need);
    hipStream_t s = (hipStream_t)stream;
    const int K = p->K;
    if (!p->d_objs) HIP_TRY(hipMalloc(&p->d_objs, sizeof(PaperObj) * K));
    if (!p->d_tab[network]) HIP_TRY(hipMalloc(&p->d_tab[network], sizeof(void*) * 4 * K));
    if (p->tab_dirty[network]) {
        std::vector<void*> tab((size_t)4 * K);
        for (int k = 0; k < K; ++k) {
            tab[k] = p->gg[network][k];
            tab[K + k] = p->gm[network][k];
            tab[2 * K + k] = p->gv[network][k];
            tab[3 * K + k] = const_cast<void*>(p->objs[k].grid[network]);
        }
        HIP_TRY(hipStreamSynchronize(s));
        HIP_TRY(hipMemcpy(p->d_tab[network], tab.data(), sizeof(void*) * tab.size(), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(p->d_objs, p->objs.data(), sizeof(PaperObj) * K, hipMemcpyHostToDevice));
        p->tab_dirty[network] = false;
    }
    const int64_t ge = paper_grid_elems(network);
    for (int k = 0; k < K; ++k) HIP_TRY(launch_paper_zero(p->gg[network][k], ge, s));
    PaperTrainArgs a{};
    a.rays = rays;
    a.ids = ids;
    a.tmax = tmax;
    a.labels = labels;
    a.n = n;
    a.objs = p->d_objs;
    a.num_objects = K;
    a.w = p->w[network];
    a.mlp_m = p->mlp_m[network];
    a.mlp_v = p->mlp_v[network];
    a.padded = p->d_master[network];
    float* const* tab = reinterpret_cast<float* const*>(p->d_tab[network]);
    a.grid_grad = tab;
    a.grid_m = tab + K;
    a.grid_v = tab + 2 * K;
    a.grid = reinterpret_cast<void* const*>(tab + 3 * K);
    a.grad_out = mlp_grad;
    a.loss_out = grad_y ? nullptr : loss;
    a.grad_y = grad_y;
    a.use_adam = adam ? 1 : 0;
    if (adam) {
        a.adam.lr = adam->lr;
        a.adam.beta1 = adam->beta1;
        a.adam.beta2 = adam->beta2;
        a.adam.eps = adam->eps;
        a.adam.bc1 = (float)(1.0 - std::pow((double)adam->beta1, step));
        a.adam.bc2 = (float)(1.0 - std::pow((double)adam->beta2, step));
    }
    HIP_TRY(launch_paper_train(network, a, ws, s));
    if (adam)
        for (bool& b : p->prepared) b = false;  // the weights changed: nif_paper_prepare packs them again
    return ok();
}

// ---------------------------------------------------------------------------
// Light importance sampling of training rays (Sec. 5 "Training").
// ---------------------------------------------------------------------------
struct nif_light {
    void* table = nullptr;
};

extern "C" nif_status nif_light_create(const float* tris, const float* radiance, int64_t num_tris, nif_light** out) {
    if (!out) return fail(NIF_ERR_INVALID_ARG, "nif_light_create: NULL out");
    *out = nullptr;
    if (!tris || !radiance) return fail(NIF_ERR_INVALID_ARG, "nif_light_create: NULL argument");
    if (num_tris < 1 || num_tris > ((int64_t)1 << 30)) return fail(NIF_ERR_INVALID_ARG, "nif_light_create: num_tris out of range");
    for (int64_t i = 0; i < 9 * num_tris; ++i)
        if (!isfinite(tris[i])) return fail(NIF_ERR_INVALID_ARG, "nif_light_create: non-finite vertex");
    void* h = nullptr;
    const char* why = nullptr;
    hipError_t e = light_create(tris, radiance, num_tris, &h, &why);
    if (why) return fail(NIF_ERR_INVALID_ARG, "nif_light_create: %s", why);
    if (e != hipSuccess) return fail(NIF_ERR_HIP, "nif_light_create: %s", hipGetErrorString(e));
    nif_light* l = new nif_light;
    l->table = h;
    *out = l;
    return ok();
}

extern "C" void nif_light_destroy(nif_light* l) {
    if (!l) return;
    light_destroy(l->table);
    delete l;
}

extern "C" nif_status nif_light_sample(const nif_light* l, const float* points, const float* u, int64_t n, float* rays,
                                       float* t_max, float* pdf, int32_t* tri, void* stream) {
    if (!l) return fail(NIF_ERR_INVALID_ARG, "nif_light_sample: NULL handle");
    if (n < 0) return fail(NIF_ERR_INVALID_ARG, "nif_light_sample: n < 0");
    if (n == 0) return ok();
    if (!points || !u || !rays || !t_max) return fail(NIF_ERR_INVALID_ARG, "nif_light_sample: NULL input or output");
    HIP_TRY(launch_light_sample(l->table, points, u, n, rays, t_max, pdf, tri, (hipStream_t)stream));
    return ok();
}

extern "C" nif_status nif_paper_train_step(nif_paper* p, int32_t network, const float* rays, const int32_t* ids,
                                           const float* tmax, const uint8_t* labels, int64_t n, int32_t step,
                                           const nif_adam* adam, float* loss, float* mlp_grad, void* ws,
                                           size_t ws_bytes, void* stream) {
    return paper_train_common(p, network, rays, ids, tmax, labels, nullptr, n, step, adam, loss, mlp_grad, ws,
                              ws_bytes, stream);
}

extern "C" nif_status nif_paper_backward(nif_paper* p, int32_t network, const float* rays, const int32_t* ids,
                                         const float* tmax, const float* grad_visibility, int64_t n, float* mlp_grad,
                                         void* ws, size_t ws_bytes, void* stream) {
    if (n > 0 && !grad_visibility) return fail(NIF_ERR_INVALID_ARG, "nif_paper_backward: NULL grad_visibility");
    return paper_train_common(p, network, rays, ids, tmax, nullptr, grad_visibility, n, 1, nullptr, nullptr, mlp_grad,
                              ws, ws_bytes, stream);
}
