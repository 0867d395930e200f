// The fused MLP on MFMA shared by the query kernels: weight packets in LDS,
// 32 queries per wave, two lanes per query (see nif_forward.hip for the work
// mapping), ReLU or leaky-ReLU hidden layers, binary32 output layer.
#pragma once

#include <hip/hip_runtime.h>

#include "nif_internal.h"

namespace nif {

#define GLOBAL __attribute__((address_space(1)))

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int FLAV> struct FT;
template <> struct FT<kF32> { static constexpr int ebytes = 4, kstep = 1; };
template <> struct FT<kBF16> { static constexpr int ebytes = 2, kstep = 8; };
template <> struct FT<kF16> { static constexpr int ebytes = 2, kstep = 8; };
template <> struct FT<kFP8> { static constexpr int ebytes = 1, kstep = 32; };

constexpr int roundup(int a, int b) { return (a + b - 1) / b * b; }

// 16-byte packets per M-tile of a layer whose halves hold kh local inputs.
constexpr int packets_for(int flav, int kh) {
    return flav == kF32   ? (kh * 4 + 15) / 16
           : flav == kFP8 ? roundup(kh, 32) / 16
                          : roundup(kh, 8) * 2 / 16;
}

// ----------------------------------------------------------------------------
// MLP on MFMA.
// ----------------------------------------------------------------------------
__device__ __forceinline__ i32x4 load_packet(const uint8_t* img, int idx) {
    return *reinterpret_cast<const i32x4*>(img + (int64_t)idx * 16);
}

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
// two floats -> packed pair, round to nearest even
__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{a, b}, bf16x2));
}
__device__ __forceinline__ uint32_t pack_f16x2(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{a, b}, f16x2));
}
// four floats in [-448, 448] -> four OCP E4M3 bytes, round to nearest even
__device__ __forceinline__ int pack_fp8x4_clamped(float a, float b, float c, float d) {
    int r = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
    return __builtin_amdgcn_cvt_pk_fp8_f32(c, d, r, true);
}
// saturated to +-448 first (the conversion itself does not saturate)
__device__ __forceinline__ int pack_fp8x4(float a, float b, float c, float d) {
    return pack_fp8x4_clamped(__builtin_amdgcn_fmed3f(a, -448.0f, 448.0f), __builtin_amdgcn_fmed3f(b, -448.0f, 448.0f),
                              __builtin_amdgcn_fmed3f(c, -448.0f, 448.0f), __builtin_amdgcn_fmed3f(d, -448.0f, 448.0f));
}
// ReLU and saturation in one step (the scale is positive): median of (x, 0, 448)
__device__ __forceinline__ int pack_fp8x4_relu(float a, float b, float c, float d) {
    return pack_fp8x4_clamped(__builtin_amdgcn_fmed3f(a, 0.0f, 448.0f), __builtin_amdgcn_fmed3f(b, 0.0f, 448.0f),
                              __builtin_amdgcn_fmed3f(c, 0.0f, 448.0f), __builtin_amdgcn_fmed3f(d, 0.0f, 448.0f));
}

// ReLU of a pair of rounded binary16 / bfloat16 values (sign and magnitude):
// as signed 16-bit integers the negative ones, -0 included, are below 0, so
// max(x, 0) keeps a non-negative value and turns the others into +0, which is
// the ReLU of the unrounded value rounded (rounding keeps the sign).
typedef short i16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ int relu_pair16(int x) {
    return __builtin_bit_cast(int, __builtin_elementwise_max(__builtin_bit_cast(i16x2, x), i16x2{0, 0}));
}

// Hidden-layer activation: 0 ReLU, 1 leaky ReLU with slope kLeakySlope.
constexpr float kLeakySlope = 0.01f;
template <int ACT>
__device__ __forceinline__ float activate(float v) {
    if constexpr (ACT == 0) return v > 0.0f ? v : 0.0f;
    return fmaxf(v, kLeakySlope * v);  // v for v >= 0, slope * v below
}

// Output of one MLP evaluation for the wave's 32 queries: z for this lane's query.
// xin: this half's layer-1 local inputs (din/2 floats, zero for inactive queries).
// PRE (16-bit operands): xpk holds those inputs already as packed pairs.
template <int FLAV, int KH1, int ACT = 0, bool PRE = false>
__device__ __forceinline__ float run_mlp(const uint8_t* img, const PackInfo& P, int hidden, const float* xin,
                                         const float* scales, int lane, const int* xpk = nullptr) {
    const int half = lane >> 5;
    f32x16 acc[2];
    // ------------------------------------------------------------------ layer 1
    {
        constexpr int PK = packets_for(FLAV, KH1);
        const uint8_t* L1 = img + P.layer_off[0];
        acc[0] = f32x16{};
        acc[1] = f32x16{};
        if constexpr (FLAV == kF32) {
#pragma unroll
            for (int p = 0; p < PK; ++p) {
#pragma unroll
                for (int mt = 0; mt < 2; ++mt) {
                    // bit-cast the whole packet: this compiler mis-reads a bit_cast
                    // of a single vector element (it takes element 0)
                    const f32x4 af = __builtin_bit_cast(f32x4, load_packet(L1, (mt * PK + p) * 64 + lane));
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int c = 4 * p + q;
                        float b = c < KH1 ? xin[c] : 0.0f;
                        acc[mt] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[q], b, acc[mt], 0, 0, 0);
                    }
                }
            }
        } else if constexpr (FLAV == kBF16 || FLAV == kF16) {
#pragma unroll
            for (int p = 0; p < PK; ++p) {
                i32x4 b4;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int c = 8 * p + 2 * q;
                    if constexpr (PRE) {
                        b4[q] = c < KH1 ? xpk[c / 2] : 0;
                    } else {
                        float v0 = c < KH1 ? xin[c] : 0.0f, v1 = c + 1 < KH1 ? xin[c + 1] : 0.0f;
                        b4[q] = (int)(FLAV == kBF16 ? pack_bf16x2(v0, v1) : pack_f16x2(v0, v1));
                    }
                }
#pragma unroll
                for (int mt = 0; mt < 2; ++mt) {
                    i32x4 a4 = load_packet(L1, (mt * PK + p) * 64 + lane);
                    if constexpr (FLAV == kBF16)
                        acc[mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a4),
                                                                          __builtin_bit_cast(bf16x8, b4), acc[mt], 0, 0, 0);
                    else
                        acc[mt] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a4),
                                                                         __builtin_bit_cast(f16x8, b4), acc[mt], 0, 0, 0);
                }
            }
        } else {  // FP8: one K-step of 32 local positions
            const float inv = 1.0f / scales[hidden + 0];
            i32x8 b8;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                float v[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int c = 4 * q + t;
                    v[t] = c < KH1 ? xin[c] * inv : 0.0f;
                }
                b8[q] = pack_fp8x4(v[0], v[1], v[2], v[3]);
            }
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                i32x4 lo = load_packet(L1, (mt * 2 + 0) * 64 + lane);
                i32x4 hi = load_packet(L1, (mt * 2 + 1) * 64 + lane);
                i32x8 a8 = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
                acc[mt] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a8, b8, acc[mt], 0, 0, 0, 0, 0, 0);
            }
        }
    }
    // ------------------------------------------------------------------ hidden layers 2..H
    for (int j = 1; j < hidden; ++j) {
        const uint8_t* Lj = img + P.layer_off[j];
        float deq = 1.0f, inv_next = 1.0f;
        if constexpr (FLAV == kFP8) {
            deq = scales[j - 1] * scales[hidden + j - 1];
            inv_next = 1.0f / scales[hidden + j];
        }
        // activations of the previous layer: local c = 16 mt + r
        // FP8: dequantise and scale for the next layer's codes in one product
        const float qs = deq * inv_next;
        float h[32];
#pragma unroll
        for (int c = 0; c < 32; ++c) {
            float v = acc[c / 16][c % 16];
            if constexpr (FLAV == kFP8) v *= qs;
            // with ReLU, 16-bit and FP8 operands take the ReLU at packing time
            h[c] = (ACT == 0 && FLAV != kF32) ? v : activate<ACT>(v);
        }
        acc[0] = f32x16{};
        acc[1] = f32x16{};
        if constexpr (FLAV == kF32) {
#pragma unroll
            for (int p = 0; p < 8; ++p) {
#pragma unroll
                for (int mt = 0; mt < 2; ++mt) {
                    const f32x4 af = __builtin_bit_cast(f32x4, load_packet(Lj, (mt * 8 + p) * 64 + lane));
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        acc[mt] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[q], h[4 * p + q], acc[mt], 0, 0, 0);
                }
            }
        } else if constexpr (FLAV == kBF16 || FLAV == kF16) {
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                i32x4 b4;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    b4[q] = (int)(FLAV == kBF16 ? pack_bf16x2(h[8 * p + 2 * q], h[8 * p + 2 * q + 1])
                                                : pack_f16x2(h[8 * p + 2 * q], h[8 * p + 2 * q + 1]));
                    if constexpr (ACT == 0) b4[q] = relu_pair16(b4[q]);
                }
#pragma unroll
                for (int mt = 0; mt < 2; ++mt) {
                    i32x4 a4 = load_packet(Lj, (mt * 4 + p) * 64 + lane);
                    if constexpr (FLAV == kBF16)
                        acc[mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a4),
                                                                          __builtin_bit_cast(bf16x8, b4), acc[mt], 0, 0, 0);
                    else
                        acc[mt] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a4),
                                                                         __builtin_bit_cast(f16x8, b4), acc[mt], 0, 0, 0);
                }
            }
        } else {
            i32x8 b8;
#pragma unroll
            for (int q = 0; q < 8; ++q)
                b8[q] = pack_fp8x4_relu(h[4 * q], h[4 * q + 1], h[4 * q + 2], h[4 * q + 3]);
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                i32x4 lo = load_packet(Lj, (mt * 2 + 0) * 64 + lane);
                i32x4 hi = load_packet(Lj, (mt * 2 + 1) * 64 + lane);
                i32x8 a8 = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
                acc[mt] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a8, b8, acc[mt], 0, 0, 0, 0, 0, 0);
            }
        }
    }
    // ------------------------------------------------------------------ output layer (binary32)
    const float* wo = reinterpret_cast<const float*>(img + P.layer_off[hidden]) + half * 32;
    float deq = 1.0f;
    if constexpr (FLAV == kFP8) deq = scales[hidden - 1] * scales[2 * hidden - 1];
    float zp = 0.0f;
#pragma unroll
    for (int c = 0; c < 32; ++c) {
        float v = acc[c / 16][c % 16];
        if constexpr (FLAV == kFP8) v *= deq;
        zp = fmaf(wo[c], activate<ACT>(v), zp);
    }
    return zp + __shfl_xor(zp, 32);
}

}  // namespace nif
