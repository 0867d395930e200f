// Weight images for the MFMA layer chain, built on the device from the
// binary32 master weights (row-major [out][in] per layer, w_out last).
//
// Forward image (any flavour): see PackInfo.  Backward image (binary32 only,
// used by the training step): per layer j, the transpose W_j^T arranged so
// that the accumulator of W_j^T . delta_j holds delta_{j-1} (or the feature
// gradient g_x for layer 1) in the lane that owns that feature in the forward
// pass.  Layout per layer: 2 M-tiles x 8 packets x 64 lanes x 4 floats
// (K = 64 output features, one per K-step and lane half).
#include <hip/hip_fp16.h>

#include "nif_internal.h"

namespace nif {

__device__ __forceinline__ uint8_t e4m3_sat(float v) {
    v = fminf(fmaxf(v, -448.0f), 448.0f);  // the conversion does not saturate by itself
    return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(v, 0.0f, 0, false) & 0xff);
}

// One thread per byte-group element of the forward image.
__global__ void pack_forward_kernel(const float* __restrict__ W, uint8_t* __restrict__ out, PackInfo P, int flav,
                                    int din, int width, const float* scales_w) {
    const int H = P.hidden;
    const int eb = flav == kF32 ? 4 : flav == kFP8 ? 1 : 2;
    const int epp = 16 / eb;
    const int64_t total_elems = P.layer_off[H] / eb;  // elements of the layer images
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total_elems + 64;
         e += (int64_t)gridDim.x * blockDim.x) {
        if (e >= total_elems) {  // w_out, permuted per half, binary32
            const int k = (int)(e - total_elems);
            const int half = k / 32, c = k % 32;
            const float* wout = W + (int64_t)width * din + (int64_t)(H - 1) * width * width;
            reinterpret_cast<float*>(out + P.layer_off[H])[k] = wout[acc_feature(half, c)];
            continue;
        }
        const int64_t byte = e * eb;
        int j = 0;
        while (j + 1 < H && byte >= P.layer_off[j + 1]) ++j;
        const int64_t rel = (byte - P.layer_off[j]) / 16;  // packet index within the layer
        const int t = (int)((byte - P.layer_off[j]) % 16) / eb;
        const int64_t layer_packets = (P.layer_off[j + 1] - P.layer_off[j]) / 16;
        const int PK = (int)(layer_packets / (2 * 64));
        const int lane = (int)(rel % 64);
        const int p = (int)((rel / 64) % PK);
        const int mt = (int)(rel / 64 / PK);
        const int kin = j == 0 ? din : width;
        const int kh = kin / 2;
        const int half = lane / 32, row = 32 * mt + lane % 32;
        const int cc = p * epp + t;
        float w = 0.0f;
        if (cc < kh) {
            const int col = j == 0 ? half * kh + cc : acc_feature(half, cc);
            const float* Wj = W + (j == 0 ? 0 : (int64_t)width * din + (int64_t)(j - 1) * width * width);
            w = Wj[(int64_t)row * kin + col];
        }
        uint8_t* dst = out + byte;
        if (flav == kF32) {
            *reinterpret_cast<float*>(dst) = w;
        } else if (flav == kBF16) {
            __bf16 b = (__bf16)w;
            *reinterpret_cast<uint16_t*>(dst) = __builtin_bit_cast(uint16_t, b);
        } else if (flav == kF16) {
            _Float16 h = (_Float16)w;
            *reinterpret_cast<uint16_t*>(dst) = __builtin_bit_cast(uint16_t, h);
        } else {
            *dst = e4m3_sat(w / scales_w[j]);
        }
    }
}

size_t backward_image_bytes(int hidden) { return (size_t)hidden * 2 * 8 * 64 * 16; }

__global__ void pack_backward_kernel(const float* __restrict__ W, float* __restrict__ out, int hidden, int din,
                                     int width) {
    const int64_t per_layer = 2 * 8 * 64 * 4;  // floats
    const int64_t total = per_layer * hidden;
    const int kh1 = din / 2;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(e / per_layer);  // 0-based layer
        const int64_t r = e % per_layer;
        const int t = (int)(r % 4);
        const int lane = (int)((r / 4) % 64);
        const int p = (int)((r / 256) % 8);
        const int mt = (int)(r / 2048);
        const int s = 4 * p + t;                             // K-step: output feature position
        const int g = acc_feature(lane / 32, s);             // output feature of layer j
        const int row = 32 * mt + lane % 32;                 // accumulator row = input feature slot
        float w = 0.0f;
        if (j == 0) {
            // accumulator row -> (register r, lane half h) -> this half's local feature c
            const int rho = row % 32;
            const int rr = 4 * (rho / 8) + rho % 4;
            const int hh = (rho % 8) / 4;
            const int c = 16 * mt + rr;
            if (c < kh1) w = W[(int64_t)g * din + hh * kh1 + c];
        } else {
            const float* Wj = W + (int64_t)width * din + (int64_t)(j - 1) * width * width;
            w = Wj[(int64_t)g * width + row];
        }
        out[e] = w;
    }
}

hipError_t launch_pack_forward(const float* W, uint8_t* out, const PackInfo& P, int flav, int din, int width,
                               const float* scales_w, hipStream_t s) {
    const int eb = flav == kF32 ? 4 : flav == kFP8 ? 1 : 2;
    const int64_t n = P.layer_off[P.hidden] / eb + 64;
    hipLaunchKernelGGL(pack_forward_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, W, out, P, flav, din,
                       width, scales_w);
    return hipGetLastError();
}

hipError_t launch_pack_backward(const float* W, float* out, int hidden, int din, int width, hipStream_t s) {
    const int64_t n = (int64_t)hidden * 2 * 8 * 64 * 4;
    hipLaunchKernelGGL(pack_backward_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, W, out, hidden, din,
                       width);
    return hipGetLastError();
}

}  // namespace nif
