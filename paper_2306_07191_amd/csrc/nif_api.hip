// Host runtime of libnif.so: the C ABI declared in include/nif.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

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
};

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
};

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
    c->objs.resize(num_objects);
    c->masters.assign(num_mlps, nullptr);
    c->fp8.resize(num_mlps);
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
    if (!c || !aabb || !grid) return fail(NIF_ERR_INVALID_ARG, "nif_set_object: NULL argument");
    if (obj < 0 || obj >= c->K) return fail(NIF_ERR_INVALID_ARG, "object %d out of range [0, %d)", obj, c->K);
    if (mlp_index < 0 || mlp_index >= c->M) return fail(NIF_ERR_INVALID_ARG, "mlp %d out of range", mlp_index);
    for (int a = 0; a < 3; ++a) {
        if (!isfinite(aabb[a]) || !isfinite(aabb[3 + a]) || !(aabb[3 + a] > aabb[a]))
            return fail(NIF_ERR_INVALID_ARG, "object %d: AABB must be finite with hi > lo on every axis", obj);
    }
    ObjHost& o = c->objs[obj];
    memcpy(o.aabb, aabb, sizeof o.aabb);
    o.grid = grid;
    o.mlp = mlp_index;
    o.set = true;
    invalidate(c);
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
    if (!isfinite(amp) || amp < 0.0f) return fail(NIF_ERR_INVALID_ARG, "amp must be finite and >= 0");
    HIP_TRY(launch_init_grid(c->objs[obj].grid, c->d.grid_dtype, c->grid_elems, seed, (uint64_t)obj, amp,
                             (hipStream_t)stream));
    return ok();
}

// ---------------------------------------------------------------------------
// weight packing (see PackInfo)
// ---------------------------------------------------------------------------
static uint16_t bf16_rne(float f) {
    uint32_t b;
    memcpy(&b, &f, 4);
    if ((b & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
    b += 0x7fffu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}
static uint16_t f16_rne(float f) {
    _Float16 h = (_Float16)f;
    uint16_t b;
    memcpy(&b, &h, 2);
    return b;
}
// OCP E4M3: bias 7, largest finite 448, no infinity; round to nearest even, saturate
static uint8_t e4m3_rne_sat(float f) {
    uint8_t s = signbit(f) ? 0x80 : 0;
    double a = fabs((double)f);
    if (a != a) return 0x7f;
    if (a >= 448.0) return s | 0x7e;
    if (a < ldexp(1.0, -6)) {
        double m = nearbyint(a / ldexp(1.0, -9));  // subnormal step 2^-9; m == 8 encodes 2^-6
        return s | (uint8_t)m;
    }
    int e;
    frexp(a, &e);
    e -= 1;  // 2^e <= a < 2^(e+1)
    double m = nearbyint(a / ldexp(1.0, e - 3));  // 8..16
    if (m >= 16.0) {
        m = 8.0;
        e += 1;
    }
    if (e > 8 || (e == 8 && m > 14.0)) return s | 0x7e;
    return s | (uint8_t)(((e + 7) << 3) | ((int)m - 8));
}

static int hidden_feature(int half, int c) { return 32 * (c / 16) + 8 * ((c % 16) / 4) + 4 * half + (c % 4); }

static void pack_mlp(const nif_ctx* c, int flav, const float* W, const float* scales, uint8_t* out) {
    const PackInfo& P = c->pack[flav];
    const int H = c->d.hidden_layers, Wd = c->d.width, din = c->din;
    const int eb = flav == kF32 ? 4 : flav == kFP8 ? 1 : 2;
    const int epp = 16 / eb;
    memset(out, 0, P.bytes);
    for (int j = 0; j < H; ++j) {
        const int kin = j == 0 ? din : Wd;
        const int kh = kin / 2;
        const float* Wj = W + (j == 0 ? 0 : (int64_t)Wd * din + (int64_t)(j - 1) * Wd * Wd);
        const int64_t layer_bytes = P.layer_off[j + 1] - P.layer_off[j];
        const int PK = (int)(layer_bytes / (2 * 64 * 16));
        for (int mt = 0; mt < 2; ++mt)
            for (int p = 0; p < PK; ++p)
                for (int lane = 0; lane < 64; ++lane) {
                    const int half = lane / 32, row = 32 * mt + lane % 32;
                    uint8_t* dst = out + P.layer_off[j] + ((int64_t)(mt * PK + p) * 64 + lane) * 16;
                    for (int t = 0; t < epp; ++t) {
                        const int cc = p * epp + t;
                        float w = 0.0f;
                        if (cc < kh) {
                            const int col = j == 0 ? half * kh + cc : hidden_feature(half, cc);
                            w = Wj[(int64_t)row * kin + col];
                        }
                        if (flav == kF32) {
                            memcpy(dst + 4 * t, &w, 4);
                        } else if (flav == kBF16) {
                            uint16_t b = bf16_rne(w);
                            memcpy(dst + 2 * t, &b, 2);
                        } else if (flav == kF16) {
                            uint16_t b = f16_rne(w);
                            memcpy(dst + 2 * t, &b, 2);
                        } else {
                            dst[t] = e4m3_rne_sat(w / scales[j]);
                        }
                    }
                }
    }
    const float* wout = W + (int64_t)Wd * din + (int64_t)(H - 1) * Wd * Wd;
    float* wo = reinterpret_cast<float*>(out + P.layer_off[H]);
    for (int half = 0; half < 2; ++half)
        for (int cc = 0; cc < 32; ++cc) wo[half * 32 + cc] = wout[hidden_feature(half, cc)];
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
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipStreamSynchronize(s));
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
    }
    if (!c->d_objs) HIP_TRY(hipMalloc(&c->d_objs, sizeof(ObjDev) * c->K));
    HIP_TRY(hipMemcpy(c->d_objs, od.data(), sizeof(ObjDev) * c->K, hipMemcpyHostToDevice));
    // weights
    const int flav = dtype;
    const PackInfo& P = c->pack[flav];
    if (!c->d_packed[flav]) HIP_TRY(hipMalloc(&c->d_packed[flav], (size_t)P.bytes * c->M));
    std::vector<float> W(c->P);
    std::vector<uint8_t> img(P.bytes);
    for (int m = 0; m < c->M; ++m) {
        HIP_TRY(hipMemcpy(W.data(), c->masters[m], sizeof(float) * c->P, hipMemcpyDeviceToHost));
        pack_mlp(c, flav, W.data(), flav == kFP8 ? c->fp8[m].data() : nullptr, img.data());
        HIP_TRY(hipMemcpy(c->d_packed[flav] + (int64_t)m * P.bytes, img.data(), P.bytes, hipMemcpyHostToDevice));
    }
    if (flav == kFP8) {
        const int H = c->d.hidden_layers;
        std::vector<float> sc((size_t)2 * H * c->M);
        for (int m = 0; m < c->M; ++m) memcpy(&sc[(size_t)2 * H * m], c->fp8[m].data(), sizeof(float) * 2 * H);
        if (!c->d_scales) HIP_TRY(hipMalloc(&c->d_scales, sizeof(float) * sc.size()));
        HIP_TRY(hipMemcpy(c->d_scales, sc.data(), sizeof(float) * sc.size(), hipMemcpyHostToDevice));
    }
    c->prepared[flav] = true;
    return ok();
}

extern "C" size_t nif_workspace_bytes(const nif_ctx* c, int64_t n, int32_t mode) {
    if (!c || n <= 0) return 0;
    (void)mode;
    return uses_order(c, n) ? order_workspace_bytes(n, c->K) : 0;
}

extern "C" nif_status nif_set_option(nif_ctx* c, int32_t option, int64_t value) {
    if (!c) return fail(NIF_ERR_INVALID_ARG, "nif_set_option: NULL context");
    switch (option) {
    case NIF_OPT_ORDER:
        if (value < 0 || value > 2) return fail(NIF_ERR_INVALID_ARG, "NIF_OPT_ORDER takes 0, 1 or 2");
        c->order_mode = (int32_t)value;
        return ok();
    }
    return fail(NIF_ERR_INVALID_ARG, "unknown option %d", option);
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

static nif_status run_query(nif_ctx* c, int32_t dtype, const float* rays, const int32_t* ids, const float* tmax,
                            const uint32_t* perm, int64_t n, float* vis, float* logits, hipStream_t s) {
    FwdArgs a{};
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

static nif_status run_order(nif_ctx* c, const float* rays, const int32_t* ids, const float* tmax, int64_t n,
                            uint32_t* perm_dst, void* ws, const uint32_t** perm, hipStream_t s) {
    OrderArgs o{};
    o.rays = rays;
    o.ids = ids;
    o.tmax = tmax;
    o.n = n;
    o.objs = c->d_objs;
    o.num_objects = c->K;
    o.perm = perm_dst;
    HIP_TRY(launch_order(o, ws, s, perm));
    return ok();
}

extern "C" nif_status nif_query(nif_ctx* c, int32_t dtype, const float* rays, const int32_t* ids, const float* tmax,
                                int64_t n, float* vis, float* logits, void* ws, size_t ws_bytes, void* stream) {
    nif_status st = check_query_args(c, dtype, rays, ids, tmax, n, vis, "nif_query");
    if (st != NIF_OK || n == 0) return st == NIF_OK ? ok() : st;
    const size_t need = nif_workspace_bytes(c, n, 0);
    if (ws_bytes < need || (need > 0 && !ws)) return fail(NIF_ERR_WORKSPACE, "workspace too small: need %zu bytes", need);
    if (!c->prepared[dtype]) return fail(NIF_ERR_STATE, "context not prepared for dtype %d", dtype);
    const uint32_t* perm = nullptr;
    if (need > 0) {
        st = run_order(c, rays, ids, tmax, n, nullptr, ws, &perm, (hipStream_t)stream);
        if (st != NIF_OK) return st;
    }
    return run_query(c, dtype, rays, ids, tmax, perm, n, vis, logits, (hipStream_t)stream);
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
    return run_order(c, rays, ids, tmax, n, perm, ws, &p, (hipStream_t)stream);
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
    a.objs = c->d_objs;
    a.num_objects = c->K;
    a.hidden = c->d.hidden_layers;
    for (int k = 0; k < 3 * c->d.levels; ++k) a.toff[k] = c->toff[k];
    for (int l = 0; l < c->d.levels; ++l) a.res[l] = c->res[l];
}

extern "C" nif_status nif_encode(nif_ctx* c, const float* rays, const int32_t* ids, const float* tmax, int64_t n,
                                 float* features, int32_t* status, void* stream) {
    if (!c) return fail(NIF_ERR_INVALID_ARG, "nif_encode: NULL context");
    if (n < 0) return fail(NIF_ERR_INVALID_ARG, "nif_encode: n < 0");
    if (n == 0) return ok();
    if (!rays || !ids || !tmax || !features) return fail(NIF_ERR_INVALID_ARG, "nif_encode: NULL input or output");
    if (n > (int64_t)1 << 36) return fail(NIF_ERR_UNSUPPORTED, "nif_encode: n too large");
    if (!c->d_objs) return fail(NIF_ERR_STATE, "context not prepared");
    FwdArgs a{};
    fill_common(c, a);
    a.rays = rays;
    a.ids = ids;
    a.tmax = tmax;
    a.n = n;
    a.features = features;
    a.status_out = status;
    a.pack = c->pack[kF32];
    HIP_TRY(launch_encode(c->d.levels, c->d.grid_dtype, a, c->num_cus, (hipStream_t)stream));
    return ok();
}

extern "C" nif_status nif_mlp(nif_ctx* c, int32_t dtype, int32_t mlp, const float* features, int64_t n,
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
    a.features = const_cast<float*>(features);
    a.fixed_mlp = mlp;
    a.logit = logits;
    a.vis = nullptr;
    a.packed = c->d_packed[dtype];
    a.pack = c->pack[dtype];
    a.fp8_scales = dtype == kFP8 ? c->d_scales : nullptr;
    HIP_TRY(launch_mlp(dtype, c->d.levels, a, c->num_cus, (hipStream_t)stream));
    return ok();
}

extern "C" size_t nif_touched_bytes(const nif_ctx* c) {
    if (!c) return 0;
    const int64_t vertices = c->grid_elems / c->d.feats;
    return (size_t)((vertices + 31) / 32) * 4;
}

extern "C" nif_status nif_train_step(nif_ctx* c, const float* rays, const int32_t* object_ids, const float* t_max,
                                     const uint8_t* labels, int64_t n, int32_t step, const nif_adam* adam,
                                     float* const* grid_grad, float* const* grid_m, float* const* grid_v,
                                     uint32_t* const* touched, float* mlp_m, float* mlp_v, float* loss,
                                     float* mlp_grad_out, void* ws, size_t ws_bytes, void* stream) {
    (void)c; (void)rays; (void)object_ids; (void)t_max; (void)labels; (void)n; (void)step; (void)adam;
    (void)grid_grad; (void)grid_m; (void)grid_v; (void)touched; (void)mlp_m; (void)mlp_v; (void)loss;
    (void)mlp_grad_out; (void)ws; (void)ws_bytes; (void)stream;
    return fail(NIF_ERR_UNSUPPORTED, "nif_train_step: not built yet");
}
