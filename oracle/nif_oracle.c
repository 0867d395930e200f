/*
 * nif_oracle.c - plain CPU reference ("oracle") for the Neural Intersection
 * Function visibility query, its training gradient, and exact shadow-ray
 * labels.
 *
 * TEST INFRASTRUCTURE ONLY.  The product library never links, loads or calls
 * this file; only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no source, header, table or helper with the HIP
 * path.  Arithmetic is binary64 except where a floating-point result decides an
 * integer (the grid cell a point falls in): there the clip and the grid
 * coordinates are evaluated in binary32, in the order written below, because
 * that is the precision in which the GPU kernel takes the same decision.  A
 * pure binary64 variant of those steps is kept (coord_mode = 1) for the
 * error split.
 *
 * Paper: S. Fujieda, C. C. Kao, T. Harada, "Neural Intersection Function",
 * HPG 2023.  Passages followed:
 *   visibility f(p,d) in {0,1}, 0 = occluded ..................... Sec. 3, Eq. (1)
 *   a network gives a visible probability in [0,1] ................ Sec. 3
 *   replace the ray origin by its entry point on the object AABB ... Sec. 2 (end), Sec. 3.1
 *   grids of trainable latents, interpolated and concatenated ...... Sec. 3.1, Fig. 2
 *   MLP with hidden activations and a sigmoid output; occluded iff
 *   the probability is below 0.5 ................................... Sec. 5 "Architecture"
 *   query at every object AABB the ray meets ...................... Sec. 4.1
 *   latents and weights trained jointly by back-propagation ........ Sec. 3.1
 *   Adam, half latents with binary32 gradient and moments ........... Sec. 5 "Training",
 *                                                                     "Memory Footprint"
 *   initialisation of the latents U(-1e-4, 1e-4) ..................... Sec. 5 "Initialization"
 * The encoding is the multi-resolution 3D trilinear form of the paper's grid
 * lookup (entry point, exit point and direction each get L levels); the
 * readings taken where the paper is silent are listed with the design notes.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define ORC_E 3 /* encodings: entry point, exit point, direction */

/* ======================================================================
 * Number formats
 * ====================================================================== */

enum { ORC_FMT_F32 = 0, ORC_FMT_F16 = 1, ORC_FMT_BF16 = 2, ORC_FMT_E4M3 = 3 };

/* Parameters of a binary floating-point format: p significand bits (with the
 * hidden bit), smallest normal exponent, largest finite value, and whether an
 * overflow saturates (OCP FP8 E4M3 has no infinity) or goes to infinity. */
typedef struct { int p; int emin; double maxfin; int saturate; } orc_fmt;

static orc_fmt fmt_of(int f) {
    orc_fmt r;
    switch (f) {
    case ORC_FMT_F16: r.p = 11; r.emin = -14; r.maxfin = 65504.0; r.saturate = 0; break;
    case ORC_FMT_BF16: r.p = 8; r.emin = -126; r.maxfin = ldexp(255.0, 120); r.saturate = 0; break;
    case ORC_FMT_E4M3: r.p = 4; r.emin = -6; r.maxfin = 448.0; r.saturate = 1; break;
    default: r.p = 24; r.emin = -126; r.maxfin = ldexp(16777215.0, 104); r.saturate = 0; break;
    }
    return r;
}

/* Round x to the nearest value of format f, ties to even (IEEE 754
 * roundTiesToEven).  The quantum at x is 2^(max(e, emin) - p + 1) where
 * 2^e <= |x| < 2^(e+1); dividing by a power of two is exact in binary64. */
double orc_round_fmt(double x, int f) {
    if (x == 0.0 || isnan(x)) return x;
    orc_fmt F = fmt_of(f);
    double a = fabs(x);
    if (isinf(a)) return F.saturate ? copysign(F.maxfin, x) : x;
    int k;
    frexp(a, &k); /* a = m 2^k, m in [0.5, 1) */
    int e = k - 1;
    if (e < F.emin) e = F.emin;
    double q = ldexp(1.0, e - F.p + 1);
    double r = nearbyint(a / q) * q; /* default rounding mode: to nearest, ties even */
    if (r > F.maxfin) r = F.saturate ? F.maxfin : INFINITY;
    return copysign(r, x);
}

/* Distance from x to the nearest rounding boundary (midpoint between two
 * consecutive values) of format f, relative to the quantum there.  Used to
 * flag rounding decisions that a tiny perturbation could flip. */
double orc_midpoint_distance(double x, int f) {
    if (x == 0.0 || !isfinite(x)) return INFINITY;
    orc_fmt F = fmt_of(f);
    double a = fabs(x);
    int k;
    frexp(a, &k);
    int e = k - 1;
    if (e < F.emin) e = F.emin;
    double q = ldexp(1.0, e - F.p + 1);
    double s = a / q;
    double frac = s - floor(s);
    return fabs(frac - 0.5) * q; /* absolute distance to the midpoint */
}

/* IEEE 754 binary16 bits -> value. */
double orc_f16_to_f64(uint16_t h) {
    int s = h >> 15, e = (h >> 10) & 31, m = h & 1023;
    double v;
    if (e == 0) v = ldexp((double)m, -24);
    else if (e == 31) v = m ? NAN : INFINITY;
    else v = ldexp((double)(m | 1024), e - 25);
    return s ? -v : v;
}

/* bfloat16 bits (upper half of a binary32) -> value. */
double orc_bf16_to_f64(uint16_t b) {
    int s = b >> 15, e = (b >> 7) & 255, m = b & 127;
    double v;
    if (e == 0) v = ldexp((double)m, -133);
    else if (e == 255) v = m ? NAN : INFINITY;
    else v = ldexp((double)(m | 128), e - 134);
    return s ? -v : v;
}

/* OCP FP8 E4M3 ("fn": bias 7, no infinity, S.1111.111 = NaN) bits -> value. */
double orc_e4m3_to_f64(uint8_t b) {
    int s = b >> 7, e = (b >> 3) & 15, m = b & 7;
    double v;
    if (e == 15 && m == 7) v = NAN;
    else if (e == 0) v = ldexp((double)m, -9);
    else v = ldexp((double)(m | 8), e - 10);
    return s ? -v : v;
}

/* value (already representable) -> bits, for comparisons with device bytes */
uint16_t orc_f64_to_f16_bits(double x) {
    double r = orc_round_fmt(x, ORC_FMT_F16);
    uint16_t s = signbit(r) ? 0x8000 : 0;
    double a = fabs(r);
    if (isnan(r)) return 0x7e00;
    if (isinf(a)) return s | 0x7c00;
    if (a < ldexp(1.0, -14)) return s | (uint16_t)(a * ldexp(1.0, 24));
    int k;
    frexp(a, &k);
    int e = k - 1;
    uint16_t m = (uint16_t)((a / ldexp(1.0, e) - 1.0) * 1024.0);
    return s | (uint16_t)((e + 15) << 10) | m;
}

uint8_t orc_f64_to_e4m3_bits(double x) {
    if (isnan(x)) return 0x7f;
    double r = orc_round_fmt(x, ORC_FMT_E4M3);
    uint8_t s = signbit(r) ? 0x80 : 0;
    double a = fabs(r);
    if (a < ldexp(1.0, -6)) return s | (uint8_t)(a * ldexp(1.0, 9));
    int k;
    frexp(a, &k);
    int e = k - 1;
    uint8_t m = (uint8_t)((a / ldexp(1.0, e) - 1.0) * 8.0);
    return s | (uint8_t)((e + 7) << 3) | m;
}

/* ======================================================================
 * Counter-based generator for the latent initialisation
 * Philox4x64-10: J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw,
 * "Parallel Random Numbers: As Easy as 1, 2, 3", SC 2011.  Ten rounds of
 * two 64x64->128 multiplies with the round function and Weyl key schedule
 * published there.
 * ====================================================================== */

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += W0; k1 += W1; }
        unsigned __int128 p0 = (unsigned __int128)M0 * x0;
        unsigned __int128 p1 = (unsigned __int128)M1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
        x0 = y0; x1 = lo1; x2 = y2; x3 = lo0;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Initial value of element i of object obj's grid buffer: the top 24 bits m
 * of Philox word (i mod 4) at counter (i div 4, 0, 0, 0), key (seed, obj),
 * mapped to U[-amp, amp) as (m - 2^23) * (amp * 2^-23) in binary32, then
 * rounded to the storage format (the paper stores latents in half). */
float orc_init_value_f32(uint64_t seed, uint64_t obj, uint64_t i, float amp) {
    uint64_t ctr[4] = {i >> 2, 0, 0, 0}, key[2] = {seed, obj}, out[4];
    orc_philox4x64_10(ctr, key, out);
    int32_t m = (int32_t)(out[i & 3] >> 40);
    float scale = amp * 0x1p-23f; /* exact: power-of-two scaling */
    return (float)(m - (1 << 23)) * scale;
}

/* Fill [begin, begin+count) of an object's grid with the initial values. */
void orc_init_fill(uint64_t seed, uint64_t obj, float amp, int grid_dtype, int64_t begin, int64_t count,
                   void* dst) {
    for (int64_t j = 0; j < count; ++j) {
        float v = orc_init_value_f32(seed, obj, (uint64_t)(begin + j), amp);
        if (grid_dtype == 1) ((uint16_t*)dst)[j] = orc_f64_to_f16_bits((double)v);
        else ((float*)dst)[j] = v;
    }
}

/* ======================================================================
 * Model description
 * ====================================================================== */

typedef struct {
    int32_t levels, res_min, res_max, feats; /* multi-resolution grids */
    int32_t hidden, width;                   /* MLP: hidden layers of `width` */
    int32_t num_objects;
    int32_t grid_dtype; /* 0 = binary32 latents, 1 = binary16 latents */
    int32_t quant;      /* MLP arithmetic: 0 exact binary64, 1 BF16, 2 FP16, 3 FP8 E4M3 */
    int32_t coord_mode; /* 0 = clip and grid coordinates in binary32; 1 = binary64 */
    const float* aabb;  /* [num_objects][6] lo xyz, hi xyz */
    const void* const* grids; /* [num_objects]; NULL entry -> generated by orc_init_value_f32 */
    const uint64_t* grid_seed; /* [num_objects] seeds for generated grids */
    const float* grid_amp;     /* [num_objects] amplitude for generated grids */
    const int32_t* mlp_index;  /* [num_objects] */
    const double* const* mlps; /* [num_mlps] flat weights, see orc_mlp_params */
    const double* const* fp8_scales; /* [num_mlps] -> [2*hidden]: s_W,1..H then s_x,1..H */
} orc_model;

int32_t orc_din(const orc_model* m) { return ORC_E * m->levels * m->feats; }

/* W1 [width][din], W2..W_H [width][width], w_out [width]; row-major [out][in]. */
int64_t orc_mlp_params(const orc_model* m) {
    return (int64_t)m->width * orc_din(m) + (int64_t)(m->hidden - 1) * m->width * m->width + m->width;
}

/* Resolution (cells per axis) of level l: the rounded geometric progression
 * from res_min to res_max. */
void orc_level_res(int32_t levels, int32_t res_min, int32_t res_max, int32_t* res) {
    for (int l = 0; l < levels; ++l) {
        if (levels == 1) { res[l] = res_min; continue; }
        double r = res_min * pow((double)res_max / res_min, (double)l / (levels - 1));
        res[l] = (int32_t)floor(r + 0.5);
    }
}

/* Element offsets of each (encoding, level) table inside one object's grid
 * buffer: tables in order e = 0..2, l = 0..L-1, each (N+1)^3 vertices x F. */
int64_t orc_grid_offsets(const orc_model* m, int64_t* off /* [3L+1] */) {
    int32_t res[64];
    orc_level_res(m->levels, m->res_min, m->res_max, res);
    int64_t o = 0;
    for (int e = 0; e < ORC_E; ++e)
        for (int l = 0; l < m->levels; ++l) {
            off[e * m->levels + l] = o;
            int64_t v = (int64_t)(res[l] + 1) * (res[l] + 1) * (res[l] + 1);
            o += v * m->feats;
        }
    off[ORC_E * m->levels] = o;
    return o;
}

static double grid_value(const orc_model* m, int32_t obj, int64_t elem) {
    const void* g = m->grids ? m->grids[obj] : NULL;
    if (g) {
        if (m->grid_dtype == 1) return orc_f16_to_f64(((const uint16_t*)g)[elem]);
        return (double)((const float*)g)[elem];
    }
    float v = orc_init_value_f32(m->grid_seed[obj], (uint64_t)obj, (uint64_t)elem, m->grid_amp[obj]);
    if (m->grid_dtype == 1) return orc_round_fmt((double)v, ORC_FMT_F16);
    return (double)v;
}

/* ======================================================================
 * Clip and normalisation (Sec. 2 end, Sec. 3.1: encode the point where the
 * ray meets the AABB instead of its origin; an origin inside the box is its
 * own entry point).
 * The segment is [t_a, t_b] = [max(t_near, 0), min(t_far, t_max)]; the ray
 * misses the box when t_a > t_b.  Returns 1 hit, 0 miss, -1 invalid input.
 * ====================================================================== */

/* binary32 version: each operation below is one IEEE binary32 operation
 * (this file is compiled without contraction). */
static int clip32(const float o[3], const float d[3], float tmax, const float lo[3], const float hi[3],
                  float* ta, float* tb) {
    float tn = -INFINITY, tf = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0f) {
            if (o[a] < lo[a] || o[a] > hi[a]) return 0;
            continue;
        }
        float t0 = (lo[a] - o[a]) / d[a];
        float t1 = (hi[a] - o[a]) / d[a];
        float l = t0 < t1 ? t0 : t1, h = t0 < t1 ? t1 : t0;
        if (l > tn) tn = l;
        if (h < tf) tf = h;
    }
    float a0 = tn > 0.0f ? tn : 0.0f;
    float b0 = tf < tmax ? tf : tmax;
    *ta = a0;
    *tb = b0;
    return a0 <= b0 ? 1 : 0;
}

static int clip64(const double o[3], const double d[3], double tmax, const double lo[3], const double hi[3],
                  double* ta, double* tb) {
    double tn = -INFINITY, tf = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) {
            if (o[a] < lo[a] || o[a] > hi[a]) return 0;
            continue;
        }
        double t0 = (lo[a] - o[a]) / d[a], t1 = (hi[a] - o[a]) / d[a];
        double l = fmin(t0, t1), h = fmax(t0, t1);
        if (l > tn) tn = l;
        if (h < tf) tf = h;
    }
    *ta = fmax(tn, 0.0);
    *tb = fmin(tf, tmax);
    return *ta <= *tb ? 1 : 0;
}

static int valid_query(const float* r, float tmax, int32_t id, int32_t K) {
    for (int a = 0; a < 6; ++a)
        if (!isfinite(r[a])) return 0;
    if (r[3] == 0.0f && r[4] == 0.0f && r[5] == 0.0f) return 0;
    if (isnan(tmax) || tmax < 0.0f) return 0;
    if (id < 0 || id >= K) return 0;
    return 1;
}

/* clamp to [0, 1]; NaN (from an infinite segment end) maps to 0 */
static float clamp01f(float x) { return x > 0.0f ? (x < 1.0f ? x : 1.0f) : 0.0f; }
static double clamp01(double x) { return x > 0.0 ? (x < 1.0 ? x : 1.0) : 0.0; }

/* Normalised coordinates of the three encoded quantities:
 *   u[0] entry point, u[1] exit point: (p - lo) / (hi - lo), clamped to [0,1]^3
 *   u[2] direction: (d/|d| + 1) / 2.
 * In binary32 mode the values are binary32 results promoted to binary64. */
static int query_coords(const orc_model* m, const float* r, float tmax, int32_t id, double u[3][3]) {
    if (!valid_query(r, tmax, id, m->num_objects)) return -1;
    const float* bx = m->aabb + 6 * (int64_t)id;
    if (m->coord_mode == 0) {
        const float *o = r, *d = r + 3, *lo = bx, *hi = bx + 3;
        float ta, tb;
        if (!clip32(o, d, tmax, lo, hi, &ta, &tb)) return 0;
        float len2 = d[0] * d[0];
        len2 = len2 + d[1] * d[1];
        len2 = len2 + d[2] * d[2];
        float len = sqrtf(len2);
        for (int a = 0; a < 3; ++a) {
            float ext = hi[a] - lo[a];
            float pin = o[a] + ta * d[a];
            float pout = o[a] + tb * d[a];
            u[0][a] = clamp01f((pin - lo[a]) / ext);
            u[1][a] = clamp01f((pout - lo[a]) / ext);
            u[2][a] = clamp01f((d[a] / len + 1.0f) * 0.5f);
        }
        return 1;
    }
    double o[3], d[3], lo[3], hi[3];
    for (int a = 0; a < 3; ++a) { o[a] = r[a]; d[a] = r[3 + a]; lo[a] = bx[a]; hi[a] = bx[3 + a]; }
    double ta, tb;
    if (!clip64(o, d, (double)tmax, lo, hi, &ta, &tb)) return 0;
    double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int a = 0; a < 3; ++a) {
        u[0][a] = clamp01((o[a] + ta * d[a] - lo[a]) / (hi[a] - lo[a]));
        u[1][a] = clamp01((o[a] + tb * d[a] - lo[a]) / (hi[a] - lo[a]));
        u[2][a] = clamp01((d[a] / len + 1.0) * 0.5);
    }
    return 1;
}

/* ======================================================================
 * Grid encoding (Sec. 3.1, Fig. 2: latents stored at grid vertices,
 * interpolated at the query coordinate, concatenated).  Level l has N_l cells
 * per axis and (N_l+1)^3 vertices; the cell is c = min(floor(u N), N-1) and the
 * interpolation weight of corner b is prod_a (b_a ? w_a : 1 - w_a) with
 * w = u N - c.  x[(e L + l) F + f] = sum_b weight_b G[vertex_b][f].
 * Corner vertex index: ((c_z+b_z)(N+1) + c_y+b_y)(N+1) + c_x+b_x.
 * ====================================================================== */

typedef struct {
    int64_t elem[ORC_E * 16][8]; /* element index of feature 0 of each corner, per (e,l) */
    double w[ORC_E * 16][8];
} orc_corners;

static void encode(const orc_model* m, int32_t obj, double u[3][3], const int64_t* off, const int32_t* res,
                   double* x, double* gmax, orc_corners* cs) {
    const int L = m->levels, F = m->feats;
    for (int e = 0; e < ORC_E; ++e)
        for (int l = 0; l < L; ++l) {
            const int N = res[l];
            int64_t c[3];
            double w[3];
            for (int a = 0; a < 3; ++a) {
                if (m->coord_mode == 0) {
                    /* binary32: s = u N, cell = min(floor(s), N-1), w = s - cell (exact) */
                    float s = (float)u[e][a] * (float)N;
                    float cf = floorf(s);
                    if (cf > (float)(N - 1)) cf = (float)(N - 1);
                    c[a] = (int64_t)cf;
                    w[a] = (double)(s - cf);
                } else {
                    double s = u[e][a] * N;
                    double cf = floor(s);
                    if (cf > N - 1) cf = N - 1;
                    c[a] = (int64_t)cf;
                    w[a] = s - cf;
                }
            }
            const int64_t N1 = N + 1;
            for (int f = 0; f < F; ++f) {
                x[(e * L + l) * F + f] = 0.0;
                if (gmax) gmax[(e * L + l) * F + f] = 0.0;
            }
            for (int b = 0; b < 8; ++b) {
                int bx = b & 1, by = (b >> 1) & 1, bz = (b >> 2) & 1;
                int64_t v = ((c[2] + bz) * N1 + (c[1] + by)) * N1 + (c[0] + bx);
                double wt = (bx ? w[0] : 1.0 - w[0]) * (by ? w[1] : 1.0 - w[1]) * (bz ? w[2] : 1.0 - w[2]);
                int64_t el = off[e * L + l] + v * F;
                for (int f = 0; f < F; ++f) {
                    double g = grid_value(m, obj, el + f);
                    x[(e * L + l) * F + f] += wt * g;
                    if (gmax && fabs(g) > gmax[(e * L + l) * F + f]) gmax[(e * L + l) * F + f] = fabs(g);
                }
                if (cs) { cs->elem[e * L + l][b] = el; cs->w[e * L + l][b] = wt; }
            }
        }
}

/* ======================================================================
 * MLP (Sec. 5 "Architecture"): h_0 = x, h_j = act(W_j h_{j-1}) for the hidden
 * layers, z = w_out . h_H, y = sigmoid(z).  ReLU activation, no biases.
 * Optional emulation of a reduced-precision evaluation: round x and W_j
 * before each hidden layer, round h_j after the activation for j < H, keep
 * the output layer in binary32 on the unrounded h_H.  FP8 uses per-layer
 * scales: W_j ~ s_W,j q(W_j / s_W,j), h ~ s_x,j q(h / s_x,j).
 * ====================================================================== */

#define ORC_MAXW 128
#define ORC_MAXDIN 384

typedef struct {
    double z, y;
    int32_t flags;   /* rounding decisions within the drift margin of a midpoint */
    double ztol;     /* tolerance on |z_device - z|: binary32 drift plus one quantum at flagged elements */
    double ybound;   /* first-order worst-case bound on |y_device - y_exact| (exact = unquantised binary64) */
} orc_fwd;

static int qfmt(int quant) { return quant == 1 ? ORC_FMT_BF16 : quant == 2 ? ORC_FMT_F16 : ORC_FMT_E4M3; }

/* Quantum (spacing of representable values) of format f at magnitude |x|. */
static double quantum(double x, int f) {
    orc_fmt F = fmt_of(f);
    int k = 0;
    if (x != 0.0 && isfinite(x)) frexp(fabs(x), &k);
    int e = k - 1;
    if (x == 0.0 || e < F.emin) e = F.emin;
    return ldexp(1.0, e - F.p + 1);
}

/* Activation rounding of the reduced-precision path: to the format, or for
 * FP8 to scale * E4M3(h / scale) with the quotient taken in binary32. */
static double qact(double v, int quant, double scale) {
    if (quant == 3) return scale * orc_round_fmt((double)((float)v / (float)scale), ORC_FMT_E4M3);
    return orc_round_fmt(v, qfmt(quant));
}

/* Weight rounding: the binary32 master weight to the format; FP8 codes are
 * E4M3(w / s_W) with the quotient in binary32, dequantised by s_W. */
static double qweight(double w, int quant, double scale) {
    if (quant == 0) return w;
    return qact(w, quant, scale);
}

/* Largest change one rounding of a value near v can make (half a quantum,
 * times the FP8 scale). */
static double half_q(double v, int quant, double scale) {
    if (quant == 3) return 0.5 * scale * quantum(v / scale, ORC_FMT_E4M3);
    return 0.5 * quantum(v, qfmt(quant));
}

/* gamma_K = K u / (1 - K u), u = 2^-24: worst-case relative error of a
 * K-term binary32 sum of products (Higham, Accuracy and Stability of
 * Numerical Algorithms, 2nd ed., Sec. 3.1). */
static double gamma32(int K) {
    double u = ldexp(1.0, -24);
    return K * u / (1.0 - K * u);
}

#define U32 (0x1p-24)

/* Accumulation drift of one K-term dot product on the device: binary32
 * partial sums in any order, gamma_K sum|p| (Higham, Sec. 3.1).  This is the
 * model for every dtype; for FP8 operands the matrix core's internal
 * summation is not specified by a published source, so the FP8 comparison
 * with this emulation is reported, and the FP8 parity criterion is the
 * per-query bound against the unquantised binary64 result instead. */
static double acc_drift(int K, double mag) { return gamma32(K) * mag; }

/* gmax[i] = largest |latent| among the corners of feature i.  A binary32
 * evaluation of the trilinear interpolant is within 16 u gmax of the exact
 * value whether it nests linear interpolations (three levels of at most three
 * roundings of values bounded by gmax: 9 u) or sums the eight corner terms
 * (weights products of three factors 1 - w or w, each within u, formed with
 * two roundings: 5 u; an eight-term sum in any order: 8 u; 13 u in all).
 *
 * Three quantities are propagated per element:
 *   eps  worst-case bound on |device value - exact value| (Higham-style,
 *        rounding of every operand by up to half a quantum, |W| propagation)
 *   dr   drift of the device value from this emulation taking the same
 *        rounding decisions: gamma_K |terms| for the K-term binary32 sum
 *        (any summation order) plus the inputs' drift propagated in
 *        root-sum-square
 *   flip one quantum if the element's rounding decision lies within 2 dr of
 *        a midpoint (the device may round it the other way), else 0
 * ztol = 2 dr_z + sum over flagged elements of quantum x |dz/dh|. */
static void mlp_forward(const orc_model* m, const double* W, const double* sc, const double* x, const double* gmax,
                        double* acts, orc_fwd* out) {
    const int H = m->hidden, Wd = m->width, Din = orc_din(m), q = m->quant;
    double hq[ORC_MAXDIN], eps[ORC_MAXDIN], dr[ORC_MAXDIN];
    double flip[16][ORC_MAXDIN]; /* flip[j][i]: input i of layer j+1 */
    double a[ORC_MAXW], enew[ORC_MAXW], dnew[ORC_MAXW];
    double aall[17][ORC_MAXW];
    const double* Wl[17];
    int Kl[17];
    int flags = 0;
    int K = Din;
    const double s0 = (q == 3) ? sc[H] : 1.0;
    for (int i = 0; i < Din; ++i) {
        dr[i] = gmax ? 16.0 * U32 * gmax[i] : 0.0;
        hq[i] = q ? qact(x[i], q, s0) : x[i];
        eps[i] = (q ? half_q(x[i], q, s0) : 0.0) + dr[i];
        flip[0][i] = 0.0;
        if (q && orc_midpoint_distance(q == 3 ? x[i] / s0 : x[i], qfmt(q)) * (q == 3 ? s0 : 1.0) <= 2.0 * dr[i]) {
            flip[0][i] = 2.0 * half_q(x[i], q, s0);
            ++flags;
        }
    }
    const double* Wj = W;
    for (int j = 1; j <= H; ++j) {
        const double sw = (q == 3) ? sc[j - 1] : 1.0;
        Wl[j] = Wj;
        Kl[j] = K;
        for (int o = 0; o < Wd; ++o) {
            double acc = 0.0, err = 0.0, mag = 0.0, prop2 = 0.0;
            for (int i = 0; i < K; ++i) {
                double w = Wj[(int64_t)o * K + i];
                double wq = qweight(w, q, sw);
                acc += wq * hq[i];
                err += fabs(wq - w) * (fabs(hq[i]) + eps[i]) + fabs(w) * eps[i];
                mag += fabs(wq * hq[i]);
                prop2 += (wq * dr[i]) * (wq * dr[i]);
            }
            a[o] = acc;
            const double local = acc_drift(K, mag) + 1e-300;
            enew[o] = err + local;
            dnew[o] = local + sqrt(prop2);
        }
        if (acts) memcpy(acts + (int64_t)(j - 1) * Wd, a, sizeof(double) * Wd);
        memcpy(aall[j], a, sizeof(double) * Wd);
        const double sx = (q == 3 && j < H) ? sc[H + j] : 1.0;
        for (int o = 0; o < Wd; ++o) {
            double h = a[o] > 0.0 ? a[o] : 0.0;
            flip[j][o] = 0.0;
            if (j < H && q) {
                hq[o] = qact(h, q, sx);
                eps[o] = enew[o] + half_q(h + enew[o], q, sx);
                if (h > 0.0 && orc_midpoint_distance(q == 3 ? h / sx : h, qfmt(q)) * (q == 3 ? sx : 1.0) <=
                                   2.0 * dnew[o]) {
                    flip[j][o] = 2.0 * half_q(h, q, sx);
                    ++flags;
                }
            } else {
                hq[o] = h;
                eps[o] = enew[o];
            }
            dr[o] = dnew[o];
        }
        Wj += (int64_t)Wd * K;
        K = Wd;
    }
    /* output layer: binary32 on the device, unrounded h_H, binary32 w_out */
    double z = 0.0, ez = 0.0, mag = 0.0, prop2 = 0.0;
    for (int i = 0; i < Wd; ++i) {
        z += Wj[i] * hq[i];
        ez += fabs(Wj[i]) * eps[i];
        mag += fabs(Wj[i] * hq[i]);
        prop2 += (Wj[i] * dr[i]) * (Wj[i] * dr[i]);
    }
    /* first-order effect of one flipped element: its quantum times |dz/dh|,
     * with the Jacobian taken through the emulated weights and ReLU masks:
     * J_H = w_out, J_{j-1}[i] = sum_o W_j[o][i] [a_j[o] > 0] J_j[o]. */
    double tol_flip = 0.0;
    if (flags) {
        double jout[ORC_MAXDIN], jin[ORC_MAXDIN];
        for (int i = 0; i < Wd; ++i) jout[i] = Wj[i];
        for (int j = H; j >= 1; --j) {
            const double sw = (q == 3) ? sc[j - 1] : 1.0;
            for (int i = 0; i < Kl[j]; ++i) {
                double s = 0.0;
                for (int o = 0; o < Wd; ++o)
                    if (aall[j][o] > 0.0) s += qweight(Wl[j][(int64_t)o * Kl[j] + i], q, sw) * jout[o];
                jin[i] = s;
                tol_flip += flip[j - 1][i] * fabs(s);
            }
            memcpy(jout, jin, sizeof(double) * Kl[j]);
        }
    }
    out->z = z;
    out->y = 1.0 / (1.0 + exp(-z));
    out->flags = flags;
    out->ztol = 2.0 * (gamma32(Wd) * mag + sqrt(prop2)) + tol_flip;
    out->ybound = 0.25 * (ez + gamma32(Wd) * mag);
}

/* ======================================================================
 * Forward over a batch of (ray, object) queries.  Outputs (each nullable):
 *   z, y     logit and visible probability; a query that misses its AABB is
 *            visible: y = 1, z = +inf; an invalid one gives NaN
 *   status   1 hit, 0 miss, -1 invalid
 *   ztol, ybound, flags  see orc_fwd
 * ====================================================================== */

typedef struct {
    const orc_model* m;
    int64_t n;
    const float *rays, *tmax;
    const int32_t* ids;
    double *z, *y, *ztol, *ybound, *x;
    int32_t *status, *flags;
} fwd_job;

typedef void (*range_fn)(void* ctx, int64_t begin, int64_t end);
typedef struct { range_fn fn; void* ctx; int64_t b, e; } thr_arg;

static void* thr_main(void* p) {
    thr_arg* a = (thr_arg*)p;
    a->fn(a->ctx, a->b, a->e);
    return NULL;
}

int orc_default_threads(void) {
    long c = sysconf(_SC_NPROCESSORS_ONLN);
    return c > 0 ? (int)c : 1;
}

/* Run fn over [0, n) in nthreads contiguous chunks. */
static void parallel_for(int64_t n, int nthreads, range_fn fn, void* ctx) {
    if (nthreads <= 0) nthreads = orc_default_threads();
    if (nthreads > 256) nthreads = 256;
    if (n < 2 * nthreads || nthreads == 1) { fn(ctx, 0, n); return; }
    pthread_t th[256];
    thr_arg args[256];
    for (int t = 0; t < nthreads; ++t) {
        args[t].fn = fn; args[t].ctx = ctx;
        args[t].b = n * t / nthreads; args[t].e = n * (t + 1) / nthreads;
        pthread_create(&th[t], NULL, thr_main, &args[t]);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
}

static void fwd_range(void* p, int64_t b, int64_t e) {
    fwd_job* J = (fwd_job*)p;
    const orc_model* m = J->m;
    int64_t off[3 * 64 + 1];
    int32_t res[64];
    orc_grid_offsets(m, off);
    orc_level_res(m->levels, m->res_min, m->res_max, res);
    const int Din = orc_din(m);
    double x[ORC_MAXDIN], gmax[ORC_MAXDIN];
    for (int64_t i = b; i < e; ++i) {
        double u[3][3];
        const float* r = J->rays + 6 * i;
        int st = query_coords(m, r, J->tmax[i], J->ids[i], u);
        orc_fwd o = {0};
        if (st == 1) {
            int32_t obj = J->ids[i];
            encode(m, obj, u, off, res, x, gmax, NULL);
            int32_t mi = m->mlp_index[obj];
            mlp_forward(m, m->mlps[mi], m->fp8_scales ? m->fp8_scales[mi] : NULL, x, gmax, NULL, &o);
            if (J->x) memcpy(J->x + i * Din, x, sizeof(double) * Din);
        } else if (st == 0) {
            o.z = INFINITY; o.y = 1.0;
        } else {
            o.z = NAN; o.y = NAN;
        }
        if (J->z) J->z[i] = o.z;
        if (J->y) J->y[i] = o.y;
        if (J->status) J->status[i] = st;
        if (J->ztol) J->ztol[i] = o.ztol;
        if (J->ybound) J->ybound[i] = o.ybound;
        if (J->flags) J->flags[i] = o.flags;
    }
}

/* Clip status of n queries only (1: the segment meets the AABB, 0: miss,
 * -1: invalid query), the first step of orc_forward (Sec. 4.1). */
void orc_status(const orc_model* m, int64_t n, const float* rays, const int32_t* ids, const float* tmax,
                int32_t* status) {
    for (int64_t i = 0; i < n; ++i) {
        double u[3][3];
        status[i] = query_coords(m, rays + 6 * i, tmax[i], ids[i], u);
    }
}

/* Segment ends [t_a, t_b] of n queries (+inf, +inf for a miss, NaN for an
 * invalid query), in the model's coordinate precision: what the depth output
 * is measured against (t = t_a + y (t_b - t_a)). */
void orc_segment(const orc_model* m, int64_t n, const float* rays, const int32_t* ids, const float* tmax, double* ta,
                 double* tb) {
    for (int64_t i = 0; i < n; ++i) {
        const float* r = rays + 6 * i;
        ta[i] = tb[i] = NAN;
        if (!valid_query(r, tmax[i], ids[i], m->num_objects)) continue;
        const float* bx = m->aabb + 6 * (int64_t)ids[i];
        int hit;
        if (m->coord_mode == 0) {
            float a, b;
            hit = clip32(r, r + 3, tmax[i], bx, bx + 3, &a, &b);
            ta[i] = a;
            tb[i] = b;
        } else {
            double o[3], d[3], lo[3], hi[3];
            for (int k = 0; k < 3; ++k) { o[k] = r[k]; d[k] = r[3 + k]; lo[k] = bx[k]; hi[k] = bx[3 + k]; }
            hit = clip64(o, d, (double)tmax[i], lo, hi, &ta[i], &tb[i]);
        }
        if (!hit) ta[i] = tb[i] = INFINITY;
    }
}

void orc_forward(const orc_model* m, int64_t n, const float* rays, const int32_t* ids, const float* tmax,
                 double* z, double* y, int32_t* status, double* ztol, double* ybound, int32_t* flags,
                 double* x_out, int nthreads) {
    fwd_job J = {m, n, rays, tmax, ids, z, y, ztol, ybound, x_out, status, flags};
    parallel_for(n, nthreads, fwd_range, &J);
}

/* Coordinates, per-level cells and weights of one query (for tests). */
int orc_query_detail(const orc_model* m, const float* ray, int32_t id, float tmax, double* u_out /*[9]*/,
                     double* x_out /*[din]*/, int64_t* corner_elem /*[3L*8]*/, double* corner_w /*[3L*8]*/) {
    double u[3][3];
    int st = query_coords(m, ray, tmax, id, u);
    if (st != 1) return st;
    for (int e = 0; e < 3; ++e)
        for (int a = 0; a < 3; ++a) u_out[3 * e + a] = u[e][a];
    int64_t off[3 * 64 + 1];
    int32_t res[64];
    orc_grid_offsets(m, off);
    orc_level_res(m->levels, m->res_min, m->res_max, res);
    static __thread orc_corners cs;
    encode(m, id, u, off, res, x_out, NULL, &cs);
    for (int k = 0; k < ORC_E * m->levels; ++k)
        for (int b = 0; b < 8; ++b) {
            corner_elem[k * 8 + b] = cs.elem[k][b];
            corner_w[k * 8 + b] = cs.w[k][b];
        }
    return 1;
}

/* MLP alone on given inputs x [n][din] with MLP `mlp` (for tests). */
/* The MLP alone on given features; ztol / ybound (nullable) as orc_forward's
 * (no interpolation drift: the features are given). */
void orc_mlp_only(const orc_model* m, int32_t mlp, int64_t n, const double* x, double* z, double* acts, double* ztol,
                  double* ybound) {
    for (int64_t i = 0; i < n; ++i) {
        orc_fwd o;
        mlp_forward(m, m->mlps[mlp], m->fp8_scales ? m->fp8_scales[mlp] : NULL, x + i * orc_din(m), NULL,
                    acts ? acts + i * (int64_t)m->hidden * m->width : NULL, &o);
        z[i] = o.z;
        if (ztol) ztol[i] = o.ztol;
        if (ybound) ybound[i] = o.ybound;
    }
}

/* ======================================================================
 * Training gradient (Sec. 3.1: latents and weights are optimised jointly by
 * back-propagation).  Loss: binary cross-entropy on the logit, averaged over
 * the B queries of the batch that meet their AABB:
 *   L = (1/B) sum_i [softplus(z_i) - t_i z_i],  dL/dz_i = (sigmoid(z_i) - t_i) / B
 * with t_i = 1 for a visible label.  Backward through the MLP:
 *   g_wout = sum_i dz_i h_H;  delta_H = w_out dz_i * [a_H > 0]
 *   g_Wj = sum_i delta_j h_{j-1}^T;  delta_{j-1} = W_j^T delta_j * [a_{j-1} > 0]
 *   g_x = W_1^T delta_1
 * and into the grids: every corner gets g_G[vertex][f] += weight * g_x[(eL+l)F+f].
 * Exact binary64 throughout (no quantisation emulation).
 * ====================================================================== */

typedef struct {
    const orc_model* m;
    int64_t n;
    const float *rays, *tmax;
    const int32_t* ids;
    const uint8_t* labels;
    const double* grad_y; /* upstream dL/dy per query, or NULL for the BCE loss */
    double inv_b;
    int32_t num_mlps;
    double* gmlp_part; /* [nthreads][num_mlps][P] */
    double* loss_part; /* [nthreads] */
    double* gx;        /* [n][din] or NULL */
    int64_t chunk;
} bwd_job;

/* One query's gradients.  gy == NULL: binary cross-entropy against label t,
 * scaled by inv_b.  Otherwise the upstream gradient *gy = dL/dy of the
 * visibility y = sigmoid(z): dL/dz = gy sigmoid(z) (1 - sigmoid(z)). */
static void bwd_one(const orc_model* m, const double* W, const double* x, double t, double inv_b, const double* gy,
                    double* gW, double* gx, double* loss) {
    const int H = m->hidden, Wd = m->width, Din = orc_din(m);
    double h[16][ORC_MAXW > ORC_MAXDIN ? ORC_MAXW : ORC_MAXDIN];
    double a[16][ORC_MAXW];
    /* forward, keeping pre-activations a_j and activations h_j */
    memcpy(h[0], x, sizeof(double) * Din);
    const double* Wj = W;
    const double* Wl[16];
    int K = Din;
    for (int j = 1; j <= H; ++j) {
        Wl[j] = Wj;
        for (int o = 0; o < Wd; ++o) {
            double acc = 0.0;
            for (int i = 0; i < K; ++i) acc += Wj[(int64_t)o * K + i] * h[j - 1][i];
            a[j][o] = acc;
            h[j][o] = acc > 0.0 ? acc : 0.0;
        }
        Wj += (int64_t)Wd * K;
        K = Wd;
    }
    const double* wout = Wj;
    double z = 0.0;
    for (int i = 0; i < Wd; ++i) z += wout[i] * h[H][i];
    double dz;
    if (gy) {
        const double y = 1.0 / (1.0 + exp(-z));
        dz = *gy * y * (1.0 - y);
    } else {
        double sp = (z > 0.0 ? z : 0.0) + log1p(exp(-fabs(z)));
        *loss += (sp - t * z) * inv_b;
        dz = (1.0 / (1.0 + exp(-z)) - t) * inv_b;
    }
    /* output layer */
    int64_t offw[16];
    {
        int64_t o = 0;
        int KK = Din;
        for (int j = 1; j <= H; ++j) { offw[j] = o; o += (int64_t)Wd * KK; KK = Wd; }
        offw[H + 1] = o;
    }
    double delta[ORC_MAXW > ORC_MAXDIN ? ORC_MAXW : ORC_MAXDIN], dprev[ORC_MAXDIN > ORC_MAXW ? ORC_MAXDIN : ORC_MAXW];
    for (int i = 0; i < Wd; ++i) {
        gW[offw[H + 1] + i] += dz * h[H][i];
        delta[i] = a[H][i] > 0.0 ? wout[i] * dz : 0.0;
    }
    for (int j = H; j >= 1; --j) {
        int Kin = (j == 1) ? Din : Wd;
        for (int o = 0; o < Wd; ++o)
            for (int i = 0; i < Kin; ++i) gW[offw[j] + (int64_t)o * Kin + i] += delta[o] * h[j - 1][i];
        for (int i = 0; i < Kin; ++i) {
            double s = 0.0;
            for (int o = 0; o < Wd; ++o) s += Wl[j][(int64_t)o * Kin + i] * delta[o];
            dprev[i] = s;
        }
        if (j > 1)
            for (int i = 0; i < Kin; ++i) delta[i] = a[j - 1][i] > 0.0 ? dprev[i] : 0.0;
        else
            memcpy(gx, dprev, sizeof(double) * Din);
    }
}

static void bwd_range(void* p, int64_t b, int64_t e) {
    bwd_job* J = (bwd_job*)p;
    const orc_model* m = J->m;
    const int64_t P = orc_mlp_params(m);
    int tid = (int)(b / J->chunk);
    double* gpart = J->gmlp_part + (int64_t)tid * J->num_mlps * P;
    int64_t off[3 * 64 + 1];
    int32_t res[64];
    orc_grid_offsets(m, off);
    orc_level_res(m->levels, m->res_min, m->res_max, res);
    const int Din = orc_din(m);
    double x[ORC_MAXDIN], gx[ORC_MAXDIN];
    double loss = 0.0;
    for (int64_t i = b; i < e; ++i) {
        double u[3][3];
        int st = query_coords(m, J->rays + 6 * i, J->tmax[i], J->ids[i], u);
        if (st != 1) {
            if (J->gx) memset(J->gx + i * Din, 0, sizeof(double) * Din);
            continue;
        }
        int32_t obj = J->ids[i];
        encode(m, obj, u, off, res, x, NULL, NULL);
        int32_t mi = m->mlp_index[obj];
        bwd_one(m, m->mlps[mi], x, J->labels ? (J->labels[i] ? 1.0 : 0.0) : 0.0, J->inv_b,
                J->grad_y ? J->grad_y + i : NULL, gpart + (int64_t)mi * P, gx, &loss);
        if (J->gx) memcpy(J->gx + i * Din, gx, sizeof(double) * Din);
    }
    J->loss_part[tid] = loss;
}

static int64_t backward_impl(const orc_model* m, int32_t num_mlps, int64_t n, const float* rays,
                             const int32_t* ids, const float* tmax, const uint8_t* labels, const double* grad_y,
                             double* loss, double* mlp_grads, double* gx, int nthreads) {
    const int64_t P = orc_mlp_params(m);
    int32_t* st = (int32_t*)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    int64_t B = 0;
    for (int64_t i = 0; i < n; ++i) {
        double u[3][3];
        st[i] = query_coords(m, rays + 6 * i, tmax[i], ids[i], u);
        B += st[i] == 1;
    }
    free(st);
    if (nthreads <= 0) nthreads = orc_default_threads();
    if (n < 2 * nthreads) nthreads = 1;
    int64_t chunk = (n + nthreads - 1) / nthreads;
    if (chunk < 1) chunk = 1;
    int nt = (int)((n + chunk - 1) / chunk);
    if (nt < 1) nt = 1;
    bwd_job J;
    J.m = m; J.n = n; J.rays = rays; J.tmax = tmax; J.ids = ids; J.labels = labels; J.grad_y = grad_y;
    J.inv_b = B > 0 ? 1.0 / (double)B : 0.0;
    J.num_mlps = num_mlps;
    J.gmlp_part = (double*)calloc((size_t)nt * num_mlps * P, sizeof(double));
    J.loss_part = (double*)calloc((size_t)nt, sizeof(double));
    J.gx = gx;
    J.chunk = chunk;
    /* chunks aligned to `chunk` so that each worker owns one partial */
    if (nt == 1) {
        bwd_range(&J, 0, n);
    } else {
        pthread_t th[256];
        thr_arg args[256];
        for (int t = 0; t < nt; ++t) {
            args[t].fn = bwd_range; args[t].ctx = &J;
            args[t].b = t * chunk; args[t].e = (t + 1) * chunk < n ? (t + 1) * chunk : n;
            pthread_create(&th[t], NULL, thr_main, &args[t]);
        }
        for (int t = 0; t < nt; ++t) pthread_join(th[t], NULL);
    }
    memset(mlp_grads, 0, sizeof(double) * num_mlps * P);
    double L = 0.0;
    for (int t = 0; t < nt; ++t) {
        for (int64_t k = 0; k < num_mlps * P; ++k) mlp_grads[k] += J.gmlp_part[(int64_t)t * num_mlps * P + k];
        L += J.loss_part[t];
    }
    *loss = L;
    free(J.gmlp_part);
    free(J.loss_part);
    return B;
}

/* Training gradients (Sec. 4.2): binary cross-entropy on the logits, mean over
 * the B queries that meet their AABB.  Returns B.  mlp_grads: [num_mlps][P],
 * overwritten; gx: [n][din] feature gradients or NULL. */
int64_t orc_backward(const orc_model* m, int32_t num_mlps, int64_t n, const float* rays, const int32_t* ids,
                     const float* tmax, const uint8_t* labels, double* loss, double* mlp_grads, double* gx,
                     int nthreads) {
    return backward_impl(m, num_mlps, n, rays, ids, tmax, labels, NULL, loss, mlp_grads, gx, nthreads);
}

/* Gradients of sum_i grad_y[i] * y_i (chain rule through the sigmoid, the MLP
 * and the interpolation), no 1/B factor.  Returns B. */
int64_t orc_backward_given(const orc_model* m, int32_t num_mlps, int64_t n, const float* rays, const int32_t* ids,
                           const float* tmax, const double* grad_y, double* mlp_grads, double* gx, int nthreads) {
    double loss = 0.0;
    return backward_impl(m, num_mlps, n, rays, ids, tmax, NULL, grad_y, &loss, mlp_grads, gx, nthreads);
}

/* Scatter per-query feature gradients gx [n][din] into a dense binary64 grid
 * gradient of object obj (all queries with ids[i] == obj), query order. */
void orc_grid_grad_dense(const orc_model* m, int32_t obj, int64_t n, const float* rays, const int32_t* ids,
                         const float* tmax, const double* gx, double* grad) {
    int64_t off[3 * 64 + 1];
    int32_t res[64];
    orc_grid_offsets(m, off);
    orc_level_res(m->levels, m->res_min, m->res_max, res);
    const int L = m->levels, F = m->feats, Din = orc_din(m);
    double x[ORC_MAXDIN];
    static __thread orc_corners cs;
    for (int64_t i = 0; i < n; ++i) {
        if (ids[i] != obj) continue;
        double u[3][3];
        if (query_coords(m, rays + 6 * i, tmax[i], ids[i], u) != 1) continue;
        encode(m, obj, u, off, res, x, NULL, &cs);
        for (int k = 0; k < ORC_E * L; ++k)
            for (int b = 0; b < 8; ++b)
                for (int f = 0; f < F; ++f) grad[cs.elem[k][b] + f] += cs.w[k][b] * gx[i * Din + k * F + f];
    }
}

static int cmp_i64(const void* a, const void* b) {
    int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return (x > y) - (x < y);
}

/* Same sums, but only at the listed element indices (sorted ascending) of
 * object obj: out[k] = gradient at elem[k].  For grids too large to hold. */
void orc_grid_grad_at(const orc_model* m, int32_t obj, int64_t n, const float* rays, const int32_t* ids,
                      const float* tmax, const double* gx, int64_t count, const int64_t* elem, double* out) {
    int64_t off[3 * 64 + 1];
    int32_t res[64];
    orc_grid_offsets(m, off);
    orc_level_res(m->levels, m->res_min, m->res_max, res);
    const int L = m->levels, F = m->feats, Din = orc_din(m);
    double x[ORC_MAXDIN];
    static __thread orc_corners cs;
    memset(out, 0, sizeof(double) * count);
    for (int64_t i = 0; i < n; ++i) {
        if (ids[i] != obj) continue;
        double u[3][3];
        if (query_coords(m, rays + 6 * i, tmax[i], ids[i], u) != 1) continue;
        encode(m, obj, u, off, res, x, NULL, &cs);
        for (int k = 0; k < ORC_E * L; ++k)
            for (int b = 0; b < 8; ++b)
                for (int f = 0; f < F; ++f) {
                    int64_t key = cs.elem[k][b] + f;
                    const int64_t* hit = (const int64_t*)bsearch(&key, elem, count, sizeof(int64_t), cmp_i64);
                    if (hit) out[hit - elem] += cs.w[k][b] * gx[i * Din + k * F + f];
                }
    }
}

/* ======================================================================
 * Exact labels (Sec. 3, Eq. (1)): a shadow ray is visible (1) iff no triangle
 * of the object is hit at a distance t with 0 < t < t_max.
 * Ray/triangle test: the watertight algorithm of S. Woop, C. Benthin, I. Wald,
 * "Watertight Ray/Triangle Intersection", JCGT 2(1), 2013, evaluated in
 * binary64: shear the triangle into the ray's frame, take the three scaled
 * barycentric edge functions U, V, W; a hit needs them all of one sign and a
 * non-zero determinant; the distance test is done without division.
 * Double-sided.
 * ====================================================================== */

/* The same test returning the hit distance: 1 and *t = T / det (binary64) when
 * the triangle is hit with 0 < t < tmax, else 0. */
int orc_ray_tri_t(const double o[3], const double d[3], double tmax, const float* tri, double* t_out) {
    int kz = 0;
    double ad[3] = {fabs(d[0]), fabs(d[1]), fabs(d[2])};
    if (ad[1] > ad[kz]) kz = 1;
    if (ad[2] > ad[kz]) kz = 2;
    int kx = (kz + 1) % 3, ky = (kx + 1) % 3;
    if (d[kz] < 0.0) { int t = kx; kx = ky; ky = t; }
    double Sx = d[kx] / d[kz], Sy = d[ky] / d[kz], Sz = 1.0 / d[kz];
    double A[3], B[3], C[3];
    for (int a = 0; a < 3; ++a) {
        A[a] = (double)tri[a] - o[a];
        B[a] = (double)tri[3 + a] - o[a];
        C[a] = (double)tri[6 + a] - o[a];
    }
    double Ax = A[kx] - Sx * A[kz], Ay = A[ky] - Sy * A[kz];
    double Bx = B[kx] - Sx * B[kz], By = B[ky] - Sy * B[kz];
    double Cx = C[kx] - Sx * C[kz], Cy = C[ky] - Sy * C[kz];
    double U = Cx * By - Cy * Bx;
    double V = Ax * Cy - Ay * Cx;
    double W = Bx * Ay - By * Ax;
    if ((U < 0.0 || V < 0.0 || W < 0.0) && (U > 0.0 || V > 0.0 || W > 0.0)) return 0;
    double det = U + V + W;
    if (det == 0.0) return 0;
    double Az = Sz * A[kz], Bz = Sz * B[kz], Cz = Sz * C[kz];
    double T = U * Az + V * Bz + W * Cz;
    if (det < 0.0) { T = -T; det = -det; }
    /* 0 < T/det < tmax */
    if (!(T > 0.0)) return 0;
    if (!isinf(tmax) && !(T < tmax * det)) return 0;
    if (t_out) *t_out = T / det;
    return 1;
}

int orc_ray_tri(const double o[3], const double d[3], double tmax, const float* tri) {
    return orc_ray_tri_t(o, d, tmax, tri, NULL);
}

typedef struct {
    int64_t T;
    const float* tris;
    int64_t n;
    const float *rays, *tmax;
    uint8_t* vis;
} brute_job;

static void brute_range(void* p, int64_t b, int64_t e) {
    brute_job* J = (brute_job*)p;
    for (int64_t i = b; i < e; ++i) {
        const float* r = J->rays + 6 * i;
        double o[3] = {r[0], r[1], r[2]}, d[3] = {r[3], r[4], r[5]};
        uint8_t v = 1;
        for (int64_t k = 0; k < J->T; ++k)
            if (orc_ray_tri(o, d, (double)J->tmax[i], J->tris + 9 * k)) { v = 0; break; }
        J->vis[i] = v;
    }
}

void orc_anyhit_brute(int64_t T, const float* tris, int64_t n, const float* rays, const float* tmax, uint8_t* vis,
                      int nthreads) {
    brute_job J = {T, tris, n, rays, tmax, vis};
    parallel_for(n, nthreads, brute_range, &J);
}

/* Bounding volume hierarchy used only to skip triangles: median split of the
 * triangle centroids along the longest axis, leaves of at most 4 triangles.
 * Node boxes are widened by a relative margin far above binary64 rounding, and
 * the slab test accepts the closed interval, so a box is never rejected for a
 * ray that the triangle test above would report as hitting it; the BVH answer
 * is therefore identical to brute force. */
typedef struct { double lo[3], hi[3]; int64_t left, right, first, count; } orc_node;
typedef struct { int64_t T, nnodes; const float* tris; int64_t* idx; orc_node* nodes; double* cen; } orc_bvh;

static double cen_key(const orc_bvh* h, int64_t t, int axis) { return h->cen[3 * t + axis]; }

static void select_kth(orc_bvh* h, int64_t* a, int64_t n, int64_t k, int axis) {
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {
        double pv = cen_key(h, a[(lo + hi) / 2], axis);
        int64_t i = lo, j = hi;
        while (i <= j) {
            while (cen_key(h, a[i], axis) < pv) ++i;
            while (cen_key(h, a[j], axis) > pv) --j;
            if (i <= j) { int64_t t = a[i]; a[i] = a[j]; a[j] = t; ++i; --j; }
        }
        if (k <= j) hi = j;
        else if (k >= i) lo = i;
        else return;
    }
}

static int64_t build_node(orc_bvh* h, int64_t first, int64_t count) {
    int64_t id = h->nnodes++;
    orc_node* nd = &h->nodes[id];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t k = first; k < first + count; ++k) {
        const float* t = h->tris + 9 * h->idx[k];
        for (int v = 0; v < 3; ++v)
            for (int a = 0; a < 3; ++a) {
                double c = t[3 * v + a];
                if (c < lo[a]) lo[a] = c;
                if (c > hi[a]) hi[a] = c;
            }
    }
    for (int a = 0; a < 3; ++a) {
        double pad = 1e-9 * (fabs(lo[a]) + fabs(hi[a]) + (hi[a] - lo[a])) + 1e-300;
        nd->lo[a] = lo[a] - pad;
        nd->hi[a] = hi[a] + pad;
    }
    if (count <= 4) {
        nd->left = nd->right = -1; nd->first = first; nd->count = count;
        return id;
    }
    double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t k = first; k < first + count; ++k)
        for (int a = 0; a < 3; ++a) {
            double c = h->cen[3 * h->idx[k] + a];
            if (c < clo[a]) clo[a] = c;
            if (c > chi[a]) chi[a] = c;
        }
    int axis = 0;
    for (int a = 1; a < 3; ++a)
        if (chi[a] - clo[a] > chi[axis] - clo[axis]) axis = a;
    int64_t half = count / 2;
    select_kth(h, h->idx + first, count, half, axis);
    nd->first = first; nd->count = 0;
    int64_t l = build_node(h, first, half);
    int64_t r = build_node(h, first + half, count - half);
    h->nodes[id].left = l;
    h->nodes[id].right = r;
    return id;
}

orc_bvh* orc_bvh_build(int64_t T, const float* tris) {
    orc_bvh* h = (orc_bvh*)calloc(1, sizeof(orc_bvh));
    h->T = T;
    h->tris = tris;
    h->idx = (int64_t*)malloc(sizeof(int64_t) * (T > 0 ? T : 1));
    h->cen = (double*)malloc(sizeof(double) * 3 * (T > 0 ? T : 1));
    h->nodes = (orc_node*)malloc(sizeof(orc_node) * (2 * (T > 0 ? T : 1) + 1));
    for (int64_t k = 0; k < T; ++k) {
        h->idx[k] = k;
        for (int a = 0; a < 3; ++a)
            h->cen[3 * k + a] = ((double)tris[9 * k + a] + tris[9 * k + 3 + a] + tris[9 * k + 6 + a]) / 3.0;
    }
    if (T > 0) build_node(h, 0, T);
    return h;
}

void orc_bvh_free(orc_bvh* h) {
    if (!h) return;
    free(h->idx); free(h->cen); free(h->nodes); free(h);
}

static int box_hit(const orc_node* nd, const double o[3], const double d[3], double tmax) {
    double tn = 0.0, tf = tmax;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) {
            if (o[a] < nd->lo[a] || o[a] > nd->hi[a]) return 0;
            continue;
        }
        double t0 = (nd->lo[a] - o[a]) / d[a], t1 = (nd->hi[a] - o[a]) / d[a];
        double l = fmin(t0, t1), h = fmax(t0, t1);
        /* widen by a relative margin so rounding of the divisions never rejects */
        l -= 1e-9 * fabs(l);
        h += 1e-9 * fabs(h);
        if (l > tn) tn = l;
        if (h < tf) tf = h;
    }
    return tn <= tf;
}

typedef struct { const orc_bvh* h; const float *rays, *tmax; uint8_t* vis; } bvh_job;

static void bvh_range(void* p, int64_t b, int64_t e) {
    bvh_job* J = (bvh_job*)p;
    const orc_bvh* h = J->h;
    int64_t stack[128];
    for (int64_t i = b; i < e; ++i) {
        const float* r = J->rays + 6 * i;
        double o[3] = {r[0], r[1], r[2]}, d[3] = {r[3], r[4], r[5]};
        double tm = (double)J->tmax[i];
        uint8_t v = 1;
        int sp = 0;
        if (h->T > 0) stack[sp++] = 0;
        while (sp && v) {
            const orc_node* nd = &h->nodes[stack[--sp]];
            if (!box_hit(nd, o, d, tm)) continue;
            if (nd->left < 0) {
                for (int64_t k = nd->first; k < nd->first + nd->count; ++k)
                    if (orc_ray_tri(o, d, tm, h->tris + 9 * h->idx[k])) { v = 0; break; }
            } else {
                stack[sp++] = nd->left;
                stack[sp++] = nd->right;
            }
        }
        J->vis[i] = v;
    }
}

void orc_anyhit_bvh(const orc_bvh* h, int64_t n, const float* rays, const float* tmax, uint8_t* vis, int nthreads) {
    bvh_job J = {h, rays, tmax, vis};
    parallel_for(n, nthreads, bvh_range, &J);
}

/* Closest hit (primary rays; the depth of Sec. 7's primary-ray use of the
 * network): t_hit[i] = min over triangles of the hit distance T / det of the
 * test above with 0 < t < t_max, +inf when none.  Brute force, then a BVH walk
 * that prunes boxes beyond the best hit so far with the same widened slab test
 * (a box holding a closer hit is never pruned, so the minimum is the brute
 * force's, bit for bit). */
typedef struct {
    int64_t T;
    const float* tris;
    const float *rays, *tmax;
    double* t_hit;
} closest_brute_job;

static void closest_brute_range(void* p, int64_t b, int64_t e) {
    closest_brute_job* J = (closest_brute_job*)p;
    for (int64_t i = b; i < e; ++i) {
        const float* r = J->rays + 6 * i;
        double o[3] = {r[0], r[1], r[2]}, d[3] = {r[3], r[4], r[5]};
        double best = INFINITY, t;
        for (int64_t k = 0; k < J->T; ++k)
            if (orc_ray_tri_t(o, d, (double)J->tmax[i], J->tris + 9 * k, &t) && t < best) best = t;
        J->t_hit[i] = best;
    }
}

void orc_closest_brute(int64_t T, const float* tris, int64_t n, const float* rays, const float* tmax, double* t_hit,
                       int nthreads) {
    closest_brute_job J = {T, tris, rays, tmax, t_hit};
    parallel_for(n, nthreads, closest_brute_range, &J);
}

typedef struct { const orc_bvh* h; const float *rays, *tmax; double* t_hit; } closest_bvh_job;

static void closest_bvh_range(void* p, int64_t b, int64_t e) {
    closest_bvh_job* J = (closest_bvh_job*)p;
    const orc_bvh* h = J->h;
    int64_t stack[128];
    for (int64_t i = b; i < e; ++i) {
        const float* r = J->rays + 6 * i;
        double o[3] = {r[0], r[1], r[2]}, d[3] = {r[3], r[4], r[5]};
        const double tm = (double)J->tmax[i];
        double best = INFINITY, t;
        int sp = 0;
        if (h->T > 0) stack[sp++] = 0;
        while (sp) {
            const orc_node* nd = &h->nodes[stack[--sp]];
            if (!box_hit(nd, o, d, best < tm ? best : tm)) continue;
            if (nd->left < 0) {
                for (int64_t k = nd->first; k < nd->first + nd->count; ++k)
                    if (orc_ray_tri_t(o, d, tm, h->tris + 9 * h->idx[k], &t) && t < best) best = t;
            } else {
                stack[sp++] = nd->left;
                stack[sp++] = nd->right;
            }
        }
        J->t_hit[i] = best;
    }
}

void orc_closest_bvh(const orc_bvh* h, int64_t n, const float* rays, const float* tmax, double* t_hit, int nthreads) {
    closest_bvh_job J = {h, rays, tmax, t_hit};
    parallel_for(n, nthreads, closest_bvh_range, &J);
}

/* ======================================================================
 * The same watertight test evaluated in binary32, the precision the GPU
 * caster decides hits in: each operation below is one binary32 operation
 * (no contraction), and the three edge functions are recomputed in binary64
 * when one of them is exactly zero, as the published algorithm prescribes
 * for single precision.  The axis kz is the last index of the largest |d|
 * component.  Hit distance T / det in binary32.  Used to check the GPU
 * labels and closest hits decision for decision; the binary64 test above is
 * the exact reference they are also compared with.
 * ====================================================================== */
int orc_ray_tri32_t(const float o[3], const float d[3], float tmax, const float* v, float* t_out) {
    const float a0 = fabsf(d[0]), a1 = fabsf(d[1]), a2 = fabsf(d[2]);
    int kz = a0 > a1 ? (a0 > a2 ? 0 : 2) : (a1 > a2 ? 1 : 2);
    int kx = kz == 2 ? 0 : kz + 1, ky = kx == 2 ? 0 : kx + 1;
    if (d[kz] < 0.0f) { int t = kx; kx = ky; ky = t; }
    const float Sx = d[kx] / d[kz], Sy = d[ky] / d[kz], Sz = 1.0f / d[kz];
    const float Ax = v[0 + kx] - o[kx], Ay = v[0 + ky] - o[ky], Az0 = v[0 + kz] - o[kz];
    const float Bx = v[3 + kx] - o[kx], By = v[3 + ky] - o[ky], Bz0 = v[3 + kz] - o[kz];
    const float Cx = v[6 + kx] - o[kx], Cy = v[6 + ky] - o[ky], Cz0 = v[6 + kz] - o[kz];
    const float ax = Ax - Sx * Az0, ay = Ay - Sy * Az0;
    const float bx = Bx - Sx * Bz0, by = By - Sy * Bz0;
    const float cx = Cx - Sx * Cz0, cy = Cy - Sy * Cz0;
    float U = cx * by - cy * bx;
    float V = ax * cy - ay * cx;
    float W = bx * ay - by * ax;
    if (U == 0.0f || V == 0.0f || W == 0.0f) {
        U = (float)((double)cx * by - (double)cy * bx);
        V = (float)((double)ax * cy - (double)ay * cx);
        W = (float)((double)bx * ay - (double)by * ax);
    }
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return 0;
    float det = U + V + W;
    if (det == 0.0f) return 0;
    float T = U * (Sz * Az0) + V * (Sz * Bz0) + W * (Sz * Cz0);
    if (det < 0.0f) { T = -T; det = -det; }
    if (!(T > 0.0f)) return 0;
    if (!(isinf(tmax) || T < tmax * det)) return 0;
    if (t_out) *t_out = T / det;
    return 1;
}

typedef struct {
    int64_t T;
    const float* tris;
    const float *rays, *tmax;
    uint8_t* vis;
    float* t_hit;
} brute32_job;

static void brute32_range(void* p, int64_t b, int64_t e) {
    brute32_job* J = (brute32_job*)p;
    for (int64_t i = b; i < e; ++i) {
        const float* r = J->rays + 6 * i;
        float best = INFINITY, t;
        int hit = 0;
        for (int64_t k = 0; k < J->T; ++k)
            if (orc_ray_tri32_t(r, r + 3, J->tmax[i], J->tris + 9 * k, &t)) {
                hit = 1;
                if (t < best) best = t;
                if (!J->t_hit) break;
            }
        if (J->vis) J->vis[i] = hit ? 0 : 1;
        if (J->t_hit) J->t_hit[i] = best;
    }
}

/* Any-hit labels (vis, nullable) and closest-hit distances (t_hit, nullable)
 * of the binary32 test over every triangle. */
void orc_trace_brute32(int64_t T, const float* tris, int64_t n, const float* rays, const float* tmax, uint8_t* vis,
                       float* t_hit, int nthreads) {
    brute32_job J = {T, tris, rays, tmax, vis, t_hit};
    parallel_for(n, nthreads, brute32_range, &J);
}

/* The same through the BVH above, whose node boxes are widened here by a
 * relative 2^-16 (far above binary32 rounding of a hit point), so that no box
 * holding a binary32 hit is skipped and the answer equals brute force. */
static int box_hit_loose(const orc_node* nd, const double o[3], const double d[3], double tmax) {
    double tn = 0.0, tf = tmax;
    for (int a = 0; a < 3; ++a) {
        const double pad = 0x1p-16 * (fabs(nd->lo[a]) + fabs(nd->hi[a]) + fabs(o[a]));
        const double lo = nd->lo[a] - pad, hi = nd->hi[a] + pad;
        if (d[a] == 0.0) {
            if (o[a] < lo || o[a] > hi) return 0;
            continue;
        }
        double t0 = (lo - o[a]) / d[a], t1 = (hi - o[a]) / d[a];
        double l = fmin(t0, t1), h = fmax(t0, t1);
        l -= 0x1p-16 * fabs(l);
        h += 0x1p-16 * fabs(h);
        if (l > tn) tn = l;
        if (h < tf) tf = h;
    }
    return tn <= tf;
}

typedef struct { const orc_bvh* h; const float *rays, *tmax; uint8_t* vis; float* t_hit; } bvh32_job;

static void bvh32_range(void* p, int64_t b, int64_t e) {
    bvh32_job* J = (bvh32_job*)p;
    const orc_bvh* h = J->h;
    int64_t stack[128];
    for (int64_t i = b; i < e; ++i) {
        const float* r = J->rays + 6 * i;
        const double o[3] = {r[0], r[1], r[2]}, d[3] = {r[3], r[4], r[5]};
        const float tm = J->tmax[i];
        float best = INFINITY, t;
        int hit = 0, sp = 0;
        if (h->T > 0) stack[sp++] = 0;
        while (sp && !(hit && !J->t_hit)) {
            const orc_node* nd = &h->nodes[stack[--sp]];
            if (!box_hit_loose(nd, o, d, best < tm ? (double)best : (double)tm)) continue;
            if (nd->left < 0) {
                for (int64_t k = nd->first; k < nd->first + nd->count; ++k)
                    if (orc_ray_tri32_t(r, r + 3, tm, h->tris + 9 * h->idx[k], &t)) {
                        hit = 1;
                        if (t < best) best = t;
                    }
            } else {
                stack[sp++] = nd->left;
                stack[sp++] = nd->right;
            }
        }
        if (J->vis) J->vis[i] = hit ? 0 : 1;
        if (J->t_hit) J->t_hit[i] = best;
    }
}

void orc_trace_bvh32(const orc_bvh* h, int64_t n, const float* rays, const float* tmax, uint8_t* vis, float* t_hit,
                     int nthreads) {
    bvh32_job J = {h, rays, tmax, vis, t_hit};
    parallel_for(n, nthreads, bvh32_range, &J);
}
