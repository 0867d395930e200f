// Fused neural visibility query for gfx950: AABB clip, multi-resolution
// trilinear grid encoding and the MLP on MFMA, in one kernel.
//
// Method (Fujieda, Kao, Harada, "Neural Intersection Function", HPG 2023):
//  - the ray is re-parameterised by the object's AABB: its entry point replaces
//    the origin so that rays on one line encode identically (Sec. 2 end, Sec. 3.1);
//  - latents stored on grids are interpolated at the encoded coordinates and
//    concatenated as the MLP input (Sec. 3.1, Fig. 2);
//  - the MLP has ReLU hidden layers and a sigmoid output, the probability that
//    the ray is not occluded by this object (Sec. 3 Eq. (1), Sec. 5 "Architecture").
//
// Work mapping.  A wave handles 32 queries at a time, two lanes per query.
// Both lanes clip and normalise (binary32, no contraction, same operation
// order everywhere so that the grid cell a point falls in is reproducible);
// lane half h then encodes lookups h*3L/2 .. (h+1)*3L/2-1 of the 3L
// (encoding, level) tables.  Those are exactly the K-positions half h feeds to
// the first MFMA, so features never leave registers.  Each hidden layer is a
// chain of 32x32xK MFMAs (N = queries); the accumulator rows a half holds are
// fed back as its next B operand, the weight columns having been permuted to
// match at pack time.  Weights are read from LDS as one 16-byte packet per
// lane and MFMA.
#include <hip/hip_fp16.h>

#include "nif_device.h"
#include "nif_internal.h"
#include "nif_mlp.h"

namespace nif {

typedef int i32x2 __attribute__((ext_vector_type(2)));

PackInfo pack_info(int flavor, int din, int hidden) {
    PackInfo p{};
    p.din = din;
    p.hidden = hidden;
    int64_t off = 0;
    for (int j = 0; j < hidden; ++j) {
        int kh = j == 0 ? din / 2 : kWidth / 2;
        int pk = flavor == kF32 ? (kh * 4 + 15) / 16 : flavor == kFP8 ? roundup(kh, 32) / 16 : roundup(kh, 8) * 2 / 16;
        p.layer_off[j] = off;
        off += (int64_t)2 * pk * 64 * 16;
    }
    p.layer_off[hidden] = off;  // w_out: [half][32] floats
    off += 2 * 32 * 4;
    p.bytes = off;
    return p;
}

size_t lds_bytes(const PackInfo& p) { return (size_t)p.bytes; }


typedef _Float16 f16x2v __attribute__((ext_vector_type(2)));

// Cell and in-cell weight of coordinate u in [0, 1] at resolution N: s = u N
// (one binary32 product), cell = min(floor(s), N - 1), w = s - cell (exact).
// No contraction: fusing u N - cell into one FMA would use the unrounded
// product for w while the cell came from the rounded one.
__device__ __forceinline__ uint32_t cell_coord(float u, float fN, uint32_t N, float& w) {
#pragma clang fp contract(off)
    float s = u * fN;
    float cf = fminf(floorf(s), (float)(N - 1));
    w = s - cf;
    const uint32_t ci = (uint32_t)(int)cf;
    return ci < N - 1 ? ci : N - 1;  // u is in [0, 1]; kept for safety
}

// Trilinear weights of the eight cell corners, corner b = bx + 2 by + 4 bz:
// prod over axes of (b_a ? w_a : 1 - w_a), formed as ((x y) z).
__device__ __forceinline__ void corner_weights(const float w[3], float cw[8]) {
    const float x0 = 1.0f - w[0], y0 = 1.0f - w[1], z0 = 1.0f - w[2];
    const float a00 = x0 * y0, a10 = w[0] * y0, a01 = x0 * w[1], a11 = w[0] * w[1];
    cw[0] = a00 * z0;
    cw[1] = a10 * z0;
    cw[2] = a01 * z0;
    cw[3] = a11 * z0;
    cw[4] = a00 * w[2];
    cw[5] = a10 * w[2];
    cw[6] = a01 * w[2];
    cw[7] = a11 * w[2];
}

// Latent pair (f0, f1) of one vertex from a dword of two binary16 values.
__device__ __forceinline__ f16x2v half_pair(uint32_t d) { return __builtin_bit_cast(f16x2v, d); }

// The interpolated feature pair: sum of corner weight x latent over the
// corners in order 0..7 (binary32 FMAs; binary16 latents convert exactly).
__device__ __forceinline__ void interp_pairs(const float cw[8], const f16x2v g[8], float& x0, float& x1) {
    float s0 = cw[0] * (float)g[0][0], s1 = cw[0] * (float)g[0][1];
#pragma unroll
    for (int c = 1; c < 8; ++c) {
        s0 = fmaf(cw[c], (float)g[c][0], s0);
        s1 = fmaf(cw[c], (float)g[c][1], s1);
    }
    x0 = s0;
    x1 = s1;
}

// Geometry of lookup t of lane half `half`: table k, cell, weights.
template <int L>
__device__ __forceinline__ int lookup_cell(const float u[3][3], int half, int t, const FwdArgs& A, uint32_t c[3],
                                           float w[3]) {
    constexpr int NL = 3 * L / 2;
    const int k = half ? NL + t : t;
    const int e = k / L, l = k % L;
    const uint32_t N = (uint32_t)A.res[l];
    const float fN = (float)N;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float ue = e == 0 ? u[0][a] : (e == 1 ? u[1][a] : u[2][a]);
        c[a] = cell_coord(ue, fN, N, w[a]);
    }
    return k;
}

// Encode the lookups of lane half `half` from the grids: NL = 3L/2 lookups, 2
// features each, local feature c = 2 t + f.  Rows (x, x+1) of the cell at
// (y, z), (y+1, z), (y, z+1), (y+1, z+1) are one load each.  The loads of G
// lookups are issued together before their interpolation (G divides NL; the
// arithmetic does not depend on G).
template <int L, typename GT, int G>
__device__ __forceinline__ void encode_half(const float u[3][3], int half, const GLOBAL GT* grid, const FwdArgs& A,
                                            float* x) {
    constexpr int NL = 3 * L / 2;
    static_assert(NL % G == 0, "batch must divide the lookups");
    constexpr int EW = sizeof(GT) == 2 ? 1 : 2;  // dwords per vertex
#pragma unroll
    for (int t0 = 0; t0 < NL; t0 += G) {
        float w[G][3];
        uint32_t q[G][4][2 * EW];
#pragma unroll
        for (int i = 0; i < G; ++i) {
            uint32_t c[3];
            const int k = lookup_cell<L>(u, half, t0 + i, A, c, w[i]);
            const uint32_t N1 = (uint32_t)A.res[k % L] + 1;
            const uint32_t v = (c[2] * N1 + c[1]) * N1 + c[0];  // < 2^31 for N <= 1024
            const GLOBAL uint32_t* p = reinterpret_cast<const GLOBAL uint32_t*>(grid + A.toff[k]) + (uint64_t)v * EW;
            const uint32_t sy = N1 * EW, sz = N1 * N1 * EW;  // in dwords
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const GLOBAL uint32_t* pr = p;
                if (r & 1) pr += sy;
                if (r >> 1) pr += sz;
#pragma unroll
                for (int j = 0; j < 2 * EW; ++j) q[i][r][j] = pr[j];  // one 8- or 16-byte load
            }
        }
#pragma unroll
        for (int i = 0; i < G; ++i) {
            const int t = t0 + i;
            float cw[8];
            corner_weights(w[i], cw);
            if constexpr (sizeof(GT) == 2) {
                f16x2v g[8];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    g[2 * r] = half_pair(q[i][r][0]);      // (x, .)
                    g[2 * r + 1] = half_pair(q[i][r][1]);  // (x+1, .)
                }
                interp_pairs(cw, g, x[2 * t], x[2 * t + 1]);
            } else {
                float s0 = 0.0f, s1 = 0.0f;
#pragma unroll
                for (int cidx = 0; cidx < 8; ++cidx) {
                    const int r = cidx >> 1, bx = cidx & 1;
                    const float g0 = __builtin_bit_cast(float, q[i][r][2 * bx]);
                    const float g1 = __builtin_bit_cast(float, q[i][r][2 * bx + 1]);
                    s0 = cidx ? fmaf(cw[cidx], g0, s0) : cw[0] * g0;
                    s1 = cidx ? fmaf(cw[cidx], g1, s1) : cw[0] * g1;
                }
                x[2 * t] = s0;
                x[2 * t + 1] = s1;
            }
        }
    }
}

// The same lookups from the y-pair image of a binary16 grid: two 16-byte loads
// per lookup (the z and z+1 faces) instead of four row loads, same corner
// order, so the features are bit-identical to encode_half.
template <int L, int G>
__device__ __forceinline__ void encode_half_image(const float u[3][3], int half, const GLOBAL _Float16* img,
                                                  const FwdArgs& A, float* x) {
    constexpr int NL = 3 * L / 2;
    static_assert(NL % G == 0, "batch must divide the lookups");
#pragma unroll
    for (int t0 = 0; t0 < NL; t0 += G) {
        float w[G][3];
        uint32_t q[G][2][4];
#pragma unroll
        for (int i = 0; i < G; ++i) {
            uint32_t c[3];
            const int k = lookup_cell<L>(u, half, t0 + i, A, c, w[i]);
            const uint32_t N = (uint32_t)A.res[k % L], N1 = N + 1;
            const uint32_t ent = (c[2] * N + c[1]) * N1 + c[0];  // entries of 4 latents (8 bytes)
            const GLOBAL uint32_t* p = reinterpret_cast<const GLOBAL uint32_t*>(img + A.ioff[k]) + (uint64_t)ent * 2;
            const uint32_t sz = N * N1 * 2;  // one z step, in dwords
#pragma unroll
            for (int zz = 0; zz < 2; ++zz) {
                const GLOBAL uint32_t* pf = zz ? p + sz : p;
#pragma unroll
                for (int j = 0; j < 4; ++j) q[i][zz][j] = pf[j];  // one 16-byte load per face
            }
        }
#pragma unroll
        for (int i = 0; i < G; ++i) {
            float cw[8];
            corner_weights(w[i], cw);
            // face dwords: (x, y), (x, y+1), (x+1, y), (x+1, y+1) -> corners bx + 2 by + 4 bz
            f16x2v g[8];
#pragma unroll
            for (int zz = 0; zz < 2; ++zz) {
                g[4 * zz + 0] = half_pair(q[i][zz][0]);
                g[4 * zz + 2] = half_pair(q[i][zz][1]);
                g[4 * zz + 1] = half_pair(q[i][zz][2]);
                g[4 * zz + 3] = half_pair(q[i][zz][3]);
            }
            interp_pairs(cw, g, x[2 * (t0 + i)], x[2 * (t0 + i) + 1]);
        }
    }
}

// The same lookups from the z-y-pair image: entry (x, y, z) holds the latent
// pairs of (x, y, z), (x, y+1, z), (x, y, z+1), (x, y+1, z+1), so the eight
// corners of a cell are 32 contiguous bytes (entries x and x+1): two 16-byte
// loads from one cache line (except when the pair straddles a line), same
// corner order as encode_half.
template <int L, int G>
__device__ __forceinline__ void encode_half_image2(const float u[3][3], int half, const GLOBAL _Float16* img,
                                                   const FwdArgs& A, float* x) {
    constexpr int NL = 3 * L / 2;
    static_assert(NL % G == 0, "batch must divide the lookups");
#pragma unroll
    for (int t0 = 0; t0 < NL; t0 += G) {
        float w[G][3];
        uint32_t q[G][2][4];
#pragma unroll
        for (int i = 0; i < G; ++i) {
            uint32_t c[3];
            const int k = lookup_cell<L>(u, half, t0 + i, A, c, w[i]);
            const uint32_t N = (uint32_t)A.res[k % L], N1 = N + 1;
            const uint32_t ent = (c[2] * N + c[1]) * N1 + c[0];  // entries of 8 latents (16 bytes)
            const GLOBAL uint32_t* p = reinterpret_cast<const GLOBAL uint32_t*>(img + A.ioff[k]) + (uint64_t)ent * 4;
#pragma unroll
            for (int bx = 0; bx < 2; ++bx) {
                const GLOBAL uint32_t* pf = p + 4 * bx;
#pragma unroll
                for (int j = 0; j < 4; ++j) q[i][bx][j] = pf[j];  // one 16-byte load per x
            }
        }
#pragma unroll
        for (int i = 0; i < G; ++i) {
            float cw[8];
            corner_weights(w[i], cw);
            // entry dwords: (y, z), (y+1, z), (y, z+1), (y+1, z+1) -> corners bx + 2 by + 4 bz
            f16x2v g[8];
#pragma unroll
            for (int bx = 0; bx < 2; ++bx)
#pragma unroll
                for (int j = 0; j < 4; ++j) g[bx + 2 * j] = half_pair(q[i][bx][j]);
            interp_pairs(cw, g, x[2 * (t0 + i)], x[2 * (t0 + i) + 1]);
        }
    }
}

// Object id of the query in processing slot `slot` (slot < n).
__device__ __forceinline__ int32_t slot_object(const FwdArgs& A, int64_t slot) {
    const int64_t q = A.perm ? (int64_t)A.perm[slot] : slot;
    return A.qrec ? __float_as_int(A.qrec[2 * q + 1].w) : A.ids[q];
}

// ----------------------------------------------------------------------------
// The fused kernel.
// ----------------------------------------------------------------------------
// MODE 0: fused query.  MODE 1: grid stage only (writes the MLP inputs and the
// clip status).  MODE 2: inference stage only (reads MLP inputs, one MLP).
// Tile shapes of the fused kernel (chosen by the plan tuner): lookups whose
// gathers are issued together, and the waves per SIMD the register budget is
// cut for.  Shape 0 is the default.  The outputs do not depend on the shape.
constexpr int shape_batch(int SH, int NL, bool image) {
    return SH == 1 ? (image ? NL : NL / 2) : SH == 2 ? 3 : (image ? 6 : NL);
}
constexpr int shape_waves(int FLAV, int SH) { return SH == 1 ? 2 : SH == 2 ? 4 : (FLAV == kF32 ? 2 : 3); }

// End of a launch that takes its tiles from counters: every block counts
// itself out on its XCD's line, and the XCD's last block zeroes the XCD's two
// counters for the next launch on them.  Every block's final, failing fetch
// has returned its value (the block read it to stop) before the block counts
// itself out, so no fetch can follow the zeroing; all of it is device-scope
// atomics, and no fence is needed (a release fence per block would write back
// the L2).  Per-XCD counts keep the end-of-launch atomics on eight lines
// instead of one.
__device__ __forceinline__ void finish_tiles(uint32_t* ctr) {
    if (threadIdx.x != 0) return;
    const int x = blockIdx.x & 7;
    const uint32_t done = atomicAdd(ctr + (8 + x) * kTileCtrStride, 1u);
    if (done == gridDim.x / 8 - 1) {  // the grid is a multiple of 8 blocks
        atomicExch(ctr + x * kTileCtrStride, 0u);
        atomicExch(ctr + (8 + x) * kTileCtrStride, 0u);
    }
}

template <int FLAV, int L, typename GT, int MODE, int IMG, int SH>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(shape_waves(FLAV, SH)))) void nif_query_kernel(FwdArgs A) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    constexpr int KH1 = 3 * L;  // layer-1 local inputs per half: 3L/2 lookups x 2 latents
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int half = lane >> 5;
    const int qlane = lane & 31;

    // Blocks are dispatched round-robin over the 8 XCDs; each XCD takes a
    // contiguous share of the tiles so that neighbouring queries share its L2.
    // With tile counters, the XCD's blocks take the share's tiles in order from
    // the XCD's counter, so the tiles in flight on an XCD at any moment are
    // neighbours in the query order (and blocks that finish early take more);
    // without, block b takes a fixed contiguous run of the share.
    const int b = blockIdx.x;
    const int xcd = b & 7;
    const int lb = xcd * A.xcd_stride + (b >> 3);
    const int64_t t_begin = (int64_t)lb * A.num_tiles / A.tiles_per_block_num;
    const int64_t t_end = (int64_t)(lb + 1) * A.num_tiles / A.tiles_per_block_num;
    const int64_t share_begin = (int64_t)xcd * A.num_tiles / 8;
    const int64_t lim = A.tile_ctr ? (int64_t)(xcd + 1) * A.num_tiles / 8 : t_end;
    // Two slots taken in turn: the slot written by call i was last read in
    // call i - 2, before every thread passed call i - 1's barrier, so one
    // barrier per call is enough.
    __shared__ int64_t next_tile[2];
    auto tile_at = [&](int64_t i) -> int64_t {  // block-uniform: every thread calls it
        if (!A.tile_ctr) return t_begin + i;
        if (threadIdx.x == 0)
            next_tile[i & 1] = share_begin + (int64_t)atomicAdd(A.tile_ctr + xcd * kTileCtrStride, 1u);
        __syncthreads();
        return next_tile[i & 1];
    };
    const int64_t first_tile = tile_at(0);

    // MLP of the block: that of the first query of its first tile (a block
    // without tiles goes straight to the end)
    int32_t blk_mlp = A.fixed_mlp;
    if (MODE == 0 && first_tile < lim) {
        const int32_t id0 = slot_object(A, first_tile * kQueriesPerBlock);
        if (id0 >= 0 && id0 < A.num_objects) blk_mlp = A.objs[id0].mlp;
    }
    if (MODE != 1 && first_tile < lim) {
        const uint8_t* src = A.packed + (int64_t)blk_mlp * A.pack.bytes;
        const int nvec = (int)(A.pack.bytes / 16);
        for (int i = threadIdx.x; i < nvec; i += kBlock)
            reinterpret_cast<i32x4*>(smem)[i] = reinterpret_cast<const i32x4*>(src)[i];
    }
    __syncthreads();

    for (int64_t it = 0;; ++it) {
        const int64_t tile = it == 0 ? first_tile : tile_at(it);
        if (tile >= lim) break;
        const int64_t slot = tile * kQueriesPerBlock + wave * kQueriesPerWave + qlane;
        const bool inb = slot < A.n;
        const int64_t q = inb && A.perm ? (int64_t)A.perm[slot] : slot;  // the query handled here
        float o[3] = {0, 0, 0}, d[3] = {1, 0, 0};
        float tm = 0.0f;
        int32_t id = -1;
        auto load_query = [&]() {
            if (inb && MODE != 2) {
                if (A.qrec) {  // one 32-byte record instead of three arrays
                    const float4 r0 = A.qrec[2 * q], r1 = A.qrec[2 * q + 1];
                    o[0] = r0.x; o[1] = r0.y; o[2] = r0.z;
                    d[0] = r0.w; d[1] = r1.x; d[2] = r1.y;
                    tm = r1.z;
                    id = __float_as_int(r1.w);
                } else {
                    const float* r = A.rays + q * 6;
#pragma unroll
                    for (int a = 0; a < 3; ++a) { o[a] = r[a]; d[a] = r[3 + a]; }
                    tm = A.tmax[q];
                    id = A.ids[q];
                }
            }
        };
        // The tile's queries are read before the MLP check below, so that their
        // loads and the check's overlap; not for FP8, whose registers would then
        // fall to two waves per SIMD.
        constexpr bool kEarlyLoad = FLAV != kFP8;
        if constexpr (kEarlyLoad) load_query();
        if (MODE == 0 && it > 0) {
            // ordered queries change MLP at object boundaries: follow the MLP of
            // the tile's first query (a block-uniform decision)
            const int32_t id0 = slot_object(A, tile * kQueriesPerBlock);
            const int32_t m = id0 >= 0 && id0 < A.num_objects ? A.objs[id0].mlp : blk_mlp;
            if (m != blk_mlp) {
                __syncthreads();
                const uint8_t* src = A.packed + (int64_t)m * A.pack.bytes;
                const int nvec = (int)(A.pack.bytes / 16);
                for (int i = threadIdx.x; i < nvec; i += kBlock)
                    reinterpret_cast<i32x4*>(smem)[i] = reinterpret_cast<const i32x4*>(src)[i];
                __syncthreads();
                blk_mlp = m;
            }
        }
        if constexpr (!kEarlyLoad) load_query();
        // status: 1 query, 0 miss (visible), -1 invalid, -2 out of range
        int status = -2;
        float xin[KH1];
#pragma unroll
        for (int c = 0; c < KH1; ++c) xin[c] = 0.0f;
        int32_t mlp = -1;
        if (MODE == 2) {
            if (inb) {
                status = 1;
                mlp = A.fixed_mlp;
                if (A.feat16) {  // 16-bit features convert exactly; the MLP rounds them to themselves
                    const i32x2* src = reinterpret_cast<const i32x2*>(A.features) + (q * (2 * KH1) + half * KH1) / 4;
#pragma unroll
                    for (int v = 0; v < KH1 / 4; ++v) {
                        const i32x2 w = src[v];
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const uint16_t b = (uint16_t)((uint32_t)w[e / 2] >> (16 * (e % 2)));
                            xin[4 * v + e] = A.feat16 == kBF16 ? (float)__builtin_bit_cast(__bf16, b)
                                                               : (float)__builtin_bit_cast(_Float16, b);
                        }
                    }
                } else {
                    const float* src = A.features + q * (2 * KH1) + half * KH1;
#pragma unroll
                    for (int c = 0; c < KH1; ++c) xin[c] = src[c];
                }
            }
        } else if (inb) {
            const uint32_t err = query_error_bits(o, d, tm, id, A.num_objects);
            if (err) {
                status = -1;
                if (A.flags) __hip_atomic_fetch_or(A.flags, err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                const ObjDev ob = A.objs[id];
                float u[3][3];
                status = clip_normalise(o, d, tm, ob, u);
                if (status == 1) {
                    mlp = ob.mlp;
                    constexpr int NL = 3 * L / 2;
                    if constexpr (IMG == 1)
                        encode_half_image<L, shape_batch(SH, NL, true)>(u, half, (const GLOBAL _Float16*)(ob.image),
                                                                         A, xin);
                    else if constexpr (IMG == 2)
                        encode_half_image2<L, shape_batch(SH, NL, true)>(u, half, (const GLOBAL _Float16*)(ob.image),
                                                                          A, xin);
                    else
                        encode_half<L, GT, shape_batch(SH, NL, false)>(u, half, (const GLOBAL GT*)(ob.grid), A, xin);
                }
            }
        }
        if (MODE == 1) {
            if (inb && A.feat16) {  // rounded to nearest-even, as the MLP would
                i32x2* dst = reinterpret_cast<i32x2*>(A.features) + (q * (2 * KH1) + half * KH1) / 4;
#pragma unroll
                for (int v = 0; v < KH1 / 4; ++v) {
                    i32x2 w;
#pragma unroll
                    for (int e = 0; e < 2; ++e) {
                        const float a = xin[4 * v + 2 * e], b = xin[4 * v + 2 * e + 1];
                        w[e] = (int)(A.feat16 == kBF16 ? pack_bf16x2(a, b) : pack_f16x2(a, b));
                    }
                    dst[v] = w;
                }
            } else if (inb) {
                float* dst = A.features + q * (2 * KH1) + half * KH1;
#pragma unroll
                for (int c = 0; c < KH1; ++c) dst[c] = xin[c];
            }
            if (inb && half == 0 && A.status_out) A.status_out[q] = status;
            continue;
        }
        // waterfall over the distinct MLPs of the wave's queries
        float z = 0.0f;
        uint64_t pend = __ballot(status == 1);
        while (pend) {
            const int first = __builtin_ctzll(pend);
            const int m0 = __shfl(mlp, first);
            const bool mine = status == 1 && mlp == m0;
            float xb[KH1];
#pragma unroll
            for (int c = 0; c < KH1; ++c) xb[c] = mine ? xin[c] : 0.0f;
            const float* sc = A.fp8_scales ? A.fp8_scales + (int64_t)m0 * 2 * A.hidden : nullptr;
            float zz;
            if (m0 == blk_mlp)
                zz = run_mlp<FLAV, KH1>(smem, A.pack, A.hidden, xb, sc, lane);
            else
                zz = run_mlp<FLAV, KH1>(A.packed + (int64_t)m0 * A.pack.bytes, A.pack, A.hidden, xb, sc, lane);
            if (mine) z = zz;
            pend &= ~__ballot(mine);
        }
        if (inb && half == 0) {
            float y, zo;
            if (status == 1) {
                zo = z;
                y = 1.0f / (1.0f + expf(-z));
            } else if (status == 0) {
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
    if (A.tile_ctr && A.tile_ctr_reset) finish_tiles(A.tile_ctr);
}

// Inference stage on 16-bit features stored in the MLP's operand format: the
// packed pairs go to the first MFMA as they are, and each wave loads its next
// tile's features while the current tile runs.
template <int FLAV, int L>
__global__ __launch_bounds__(kBlock) void nif_mlp16_kernel(FwdArgs A) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    constexpr int KH1 = 3 * L;
    constexpr int NW = KH1 / 2;  // packed words per lane
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int half = lane >> 5;
    const int qlane = lane & 31;
    const int b = blockIdx.x;
    const int lb = (b & 7) * A.xcd_stride + (b >> 3);
    const int64_t t_begin = (int64_t)lb * A.num_tiles / A.tiles_per_block_num;
    const int64_t t_end = (int64_t)(lb + 1) * A.num_tiles / A.tiles_per_block_num;
    if (t_begin >= t_end) return;
    {
        const uint8_t* src = A.packed + (int64_t)A.fixed_mlp * A.pack.bytes;
        const int nvec = (int)(A.pack.bytes / 16);
        for (int i = threadIdx.x; i < nvec; i += kBlock)
            reinterpret_cast<i32x4*>(smem)[i] = reinterpret_cast<const i32x4*>(src)[i];
    }
    __syncthreads();
    auto load = [&](int64_t tile, int* w) {
        const int64_t q = tile * kQueriesPerBlock + wave * kQueriesPerWave + qlane;
        const i32x2* src = reinterpret_cast<const i32x2*>(A.features) + (q * (2 * KH1) + half * KH1) / 4;
#pragma unroll
        for (int v = 0; v < NW / 2; ++v) {
            const i32x2 t = q < A.n ? src[v] : i32x2{0, 0};
            w[2 * v] = t[0];
            w[2 * v + 1] = t[1];
        }
    };
    int cur[NW], nxt[NW];
    load(t_begin, nxt);
    for (int64_t tile = t_begin; tile < t_end; ++tile) {
#pragma unroll
        for (int i = 0; i < NW; ++i) cur[i] = nxt[i];
        if (tile + 1 < t_end) load(tile + 1, nxt);
        const float z = run_mlp<FLAV, KH1, 0, true>(smem, A.pack, A.hidden, nullptr, nullptr, lane, cur);
        const int64_t q = tile * kQueriesPerBlock + wave * kQueriesPerWave + qlane;
        if (q < A.n && half == 0 && A.logit) A.logit[q] = z;
    }
}

template <int FLAV, int L>
static hipError_t launch_mlp16_t(const FwdArgs& a0, int num_cus, hipStream_t s) {
    FwdArgs a = a0;
    const int64_t tiles = (a.n + kQueriesPerBlock - 1) / kQueriesPerBlock;
    int64_t blocks = (int64_t)num_cus * (a.blocks_per_cu > 0 ? a.blocks_per_cu : 16);
    if (blocks > tiles) blocks = tiles;
    blocks = (blocks + 7) / 8 * 8;
    a.num_tiles = (int32_t)tiles;
    a.tiles_per_block_num = (int32_t)blocks;
    a.xcd_stride = (int32_t)(blocks / 8);
    hipLaunchKernelGGL((nif_mlp16_kernel<FLAV, L>), dim3((unsigned)blocks), dim3(kBlock), lds_bytes(a.pack), s, a);
    return hipGetLastError();
}

hipError_t launch_mlp16(int flavor, int levels, const FwdArgs& a, int num_cus, hipStream_t s) {
    if (flavor == kBF16) return levels == 8 ? launch_mlp16_t<kBF16, 8>(a, num_cus, s) : launch_mlp16_t<kBF16, 4>(a, num_cus, s);
    if (flavor == kF16) return levels == 8 ? launch_mlp16_t<kF16, 8>(a, num_cus, s) : launch_mlp16_t<kF16, 4>(a, num_cus, s);
    return hipErrorInvalidValue;
}

// Zero tile counters of unknown content right before the launch that uses
// them (a kernel, not a memset, so that the pair can be captured into a graph).
__global__ void tile_ctr_reset_kernel(uint32_t* ctr) { ctr[threadIdx.x] = 0u; }

template <int FLAV, int L, typename GT, int MODE, int IMG, int SH>
static hipError_t launch_t(const FwdArgs& a0, int num_cus, hipStream_t s) {
    FwdArgs a = a0;
    const int64_t tiles = (a.n + kQueriesPerBlock - 1) / kQueriesPerBlock;
    // persistent-style grid: a few blocks per CU, a multiple of the 8 XCDs
    int64_t blocks = (int64_t)num_cus * (a.blocks_per_cu > 0 ? a.blocks_per_cu : 16);
    if (blocks > tiles) blocks = tiles;
    blocks = (blocks + 7) / 8 * 8;
    a.num_tiles = (int32_t)tiles;
    a.tiles_per_block_num = (int32_t)blocks;
    a.xcd_stride = (int32_t)(blocks / 8);
    if (a.tile_ctr && !a.tile_ctr_reset)  // counters of unknown content: zero them first
        hipLaunchKernelGGL(tile_ctr_reset_kernel, dim3(1), dim3(kTileCtrWords), 0, s, a.tile_ctr);
    const size_t lds = MODE == 1 ? 0 : lds_bytes(a.pack);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)nif_query_kernel<FLAV, L, GT, MODE, IMG, SH>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((nif_query_kernel<FLAV, L, GT, MODE, IMG, SH>), dim3((unsigned)blocks), dim3(kBlock), lds, s, a);
    return hipGetLastError();
}

// Shapes other than 0 exist for the fused query of 8-level binary16 grids
// (the large workloads the plan tuner serves); elsewhere shape 0 runs.
template <int FLAV, int MODE, int IMG>
static hipError_t launch_shaped(const FwdArgs& a, int num_cus, hipStream_t s) {
    if constexpr (MODE == 0) {
        if (a.shape == 1) return launch_t<FLAV, 8, _Float16, MODE, IMG, 1>(a, num_cus, s);
        if (a.shape == 2) return launch_t<FLAV, 8, _Float16, MODE, IMG, 2>(a, num_cus, s);
    }
    return launch_t<FLAV, 8, _Float16, MODE, IMG, 0>(a, num_cus, s);
}

template <int FLAV, int MODE>
static hipError_t launch_f(int levels, int grid_dtype, const FwdArgs& a, int num_cus, hipStream_t s) {
    const int img = MODE != 2 && grid_dtype == 1 ? a.use_image : 0;
    if (levels == 8) {
        if (grid_dtype == 1)
            return img == 2   ? launch_shaped<FLAV, MODE, 2>(a, num_cus, s)
                   : img == 1 ? launch_shaped<FLAV, MODE, 1>(a, num_cus, s)
                              : launch_shaped<FLAV, MODE, 0>(a, num_cus, s);
        return launch_t<FLAV, 8, float, MODE, 0, 0>(a, num_cus, s);
    }
    if (grid_dtype == 1)
        return img == 2   ? launch_t<FLAV, 4, _Float16, MODE, 2, 0>(a, num_cus, s)
               : img == 1 ? launch_t<FLAV, 4, _Float16, MODE, 1, 0>(a, num_cus, s)
                          : launch_t<FLAV, 4, _Float16, MODE, 0, 0>(a, num_cus, s);
    return launch_t<FLAV, 4, float, MODE, 0, 0>(a, num_cus, s);
}

hipError_t launch_forward(int flavor, int levels, int grid_dtype, const FwdArgs& a, int num_cus, hipStream_t s) {
    switch (flavor) {
    case kF32: return launch_f<kF32, 0>(levels, grid_dtype, a, num_cus, s);
    case kBF16: return launch_f<kBF16, 0>(levels, grid_dtype, a, num_cus, s);
    case kF16: return launch_f<kF16, 0>(levels, grid_dtype, a, num_cus, s);
    case kFP8: return launch_f<kFP8, 0>(levels, grid_dtype, a, num_cus, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_encode(int levels, int grid_dtype, const FwdArgs& a, int num_cus, hipStream_t s) {
    return launch_f<kF32, 1>(levels, grid_dtype, a, num_cus, s);
}

hipError_t launch_mlp(int flavor, int levels, const FwdArgs& a, int num_cus, hipStream_t s) {
    // the grid type is irrelevant when the features are given
    switch (flavor) {
    case kF32: return launch_f<kF32, 2>(levels, 1, a, num_cus, s);
    case kBF16: return launch_f<kBF16, 2>(levels, 1, a, num_cus, s);
    case kF16: return launch_f<kF16, 2>(levels, 1, a, num_cus, s);
    case kFP8: return launch_f<kFP8, 2>(levels, 1, a, num_cus, s);
    }
    return hipErrorInvalidValue;
}

// ----------------------------------------------------------------------------
// Latent initialisation: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC 2011).
// ----------------------------------------------------------------------------
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += W0; k1 += W1; }
        const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
        const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
        const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    }
}

__global__ void init_grid_kernel(void* grid, int grid_dtype, int64_t count, uint64_t seed, uint64_t obj, float amp) {
    const int64_t nblk = (count + 3) / 4;
    const float scale = amp * 0x1p-23f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nblk; i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t c[4] = {(uint64_t)i, 0, 0, 0};
        philox4x64_10(c, seed, obj);
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int64_t e = 4 * i + w;
            if (e >= count) break;
            const int32_t m = (int32_t)(c[w] >> 40);
            const float v = (float)(m - (1 << 23)) * scale;
            if (grid_dtype == 1)
                reinterpret_cast<__half*>(grid)[e] = __float2half_rn(v);
            else
                reinterpret_cast<float*>(grid)[e] = v;
        }
    }
}

hipError_t launch_init_grid(void* grid, int grid_dtype, int64_t count, uint64_t seed, uint64_t obj, float amp,
                            hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = ((count + 3) / 4 + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(init_grid_kernel, dim3((unsigned)blocks), dim3(256), 0, s, grid, grid_dtype, count, seed, obj,
                       amp);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// y-pair query image of a binary16 grid.
// ----------------------------------------------------------------------------
int64_t image_table_elems(int32_t N, int kind) {
    return kind == 2 ? (int64_t)(N + 1) * N * N * 8 : (int64_t)(N + 1) * N * (N + 1) * 4;
}

__global__ void build_image_kernel(const uint32_t* __restrict__ grid, uint2* __restrict__ img, int64_t toff_pairs,
                                   int64_t ioff_entries, int32_t N) {
    const int64_t N1 = N + 1;
    const int64_t entries = N1 * N * N1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < entries; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t x = i % N1, r = i / N1;
        const int64_t y = r % N, z = r / N;
        const int64_t v = (z * N1 + y) * N1 + x;  // vertex (x, y, z); its two latents are one dword
        img[ioff_entries + i] = make_uint2(grid[toff_pairs + v], grid[toff_pairs + v + N1]);
    }
}

__global__ void build_image2_kernel(const uint32_t* __restrict__ grid, uint4* __restrict__ img, int64_t toff_pairs,
                                    int64_t ioff_entries, int32_t N) {
    const int64_t N1 = N + 1;
    const int64_t entries = N1 * N * N;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < entries; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t x = i % N1, r = i / N1;
        const int64_t y = r % N, z = r / N;
        const int64_t v = (z * N1 + y) * N1 + x;  // vertex (x, y, z)
        const int64_t sz = N1 * N1;
        img[ioff_entries + i] =
            make_uint4(grid[toff_pairs + v], grid[toff_pairs + v + N1], grid[toff_pairs + v + sz],
                       grid[toff_pairs + v + sz + N1]);
    }
}

hipError_t launch_build_image(const void* grid, void* image, const int64_t* toff, const int64_t* ioff,
                              const int32_t* res, int levels, int kind, hipStream_t s) {
    for (int k = 0; k < 3 * levels; ++k) {
        const int32_t N = res[k % levels];
        if (kind == 2) {
            const int64_t entries = (int64_t)(N + 1) * N * N;
            const int64_t blocks = (entries + 255) / 256 < 65536 ? (entries + 255) / 256 : 65536;
            hipLaunchKernelGGL(build_image2_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                               reinterpret_cast<const uint32_t*>(grid), reinterpret_cast<uint4*>(image), toff[k] / 2,
                               ioff[k] / 8, N);
            continue;
        }
        const int64_t entries = (int64_t)(N + 1) * N * (N + 1);
        const int64_t blocks = (entries + 255) / 256 < 65536 ? (entries + 255) / 256 : 65536;
        // offsets in latents: the grid's 2 latents per vertex are one dword, an
        // image entry (4 latents) is 8 bytes
        hipLaunchKernelGGL(build_image_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                           reinterpret_cast<const uint32_t*>(grid), reinterpret_cast<uint2*>(image), toff[k] / 2,
                           ioff[k] / 4, N);
    }
    return hipGetLastError();
}

}  // namespace nif
