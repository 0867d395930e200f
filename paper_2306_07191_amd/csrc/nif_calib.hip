// FP8 E4M3 calibration of one MLP: the largest magnitude of every weight
// matrix W_1..W_H and of every layer input (x for layer 1, h_{j-1} for layer
// j) over a set of queries, in binary32.  The per-layer scales are these
// maxima divided by 448, the largest finite E4M3 value, so that the largest
// element of each operand lands on 448.
#include "nif_internal.h"

namespace nif {

__global__ void calib_zero_kernel(unsigned* p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

// One thread per query: binary32 forward of the layers 1..H-1 from the
// features, recording max |layer input| per layer.  A thread's layer input
// lives in LDS (column tid), its layer output in registers.  Non-negative
// binary32 values order like their bit patterns, so the maxima are kept as
// unsigned words with atomicMax.
constexpr int kCalibBlock = 128;
__global__ __launch_bounds__(kCalibBlock) void calib_act_kernel(const float* __restrict__ feats,
                                                                const int32_t* __restrict__ status,
                                                                const int32_t* __restrict__ ids,
                                                                const ObjDev* __restrict__ objs, int32_t mlp,
                                                                int64_t n, const float* __restrict__ W, int din,
                                                                int hidden, unsigned* amax) {
    __shared__ float hs[kWidth][kCalibBlock];
    const int tid = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * kCalibBlock + tid;
    const bool act = i < n && status[i] == 1 && objs[ids[i]].mlp == mlp;
    float mx0 = 0.0f;
    for (int c = 0; c < din; ++c) {
        const float v = act ? feats[i * din + c] : 0.0f;
        hs[c][tid] = v;
        mx0 = fmaxf(mx0, fabsf(v));
    }
    float mx[kMaxHidden];
    mx[0] = mx0;
#pragma unroll
    for (int j = 1; j < kMaxHidden; ++j) mx[j] = 0.0f;
    const float* Wj = W;
    int kin = din;
    for (int j = 1; j < hidden; ++j) {  // h_j = ReLU(W_j h_{j-1}), the input of layer j+1
        float o[kWidth];
#pragma unroll
        for (int r = 0; r < kWidth; ++r) o[r] = 0.0f;
        for (int c = 0; c < kin; ++c) {
            const float hc = hs[c][tid];
#pragma unroll
            for (int r = 0; r < kWidth; ++r) o[r] = fmaf(Wj[r * kin + c], hc, o[r]);
        }
        float m = 0.0f;
#pragma unroll
        for (int r = 0; r < kWidth; ++r) {
            const float v = fmaxf(o[r], 0.0f);
            hs[r][tid] = v;
            m = fmaxf(m, v);
        }
#pragma unroll
        for (int k = 1; k < kMaxHidden; ++k)
            if (k == j) mx[k] = m;
        Wj += (int64_t)kWidth * kin;
        kin = kWidth;
    }
#pragma unroll
    for (int j = 0; j < kMaxHidden; ++j) {
        float v = mx[j];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
        if ((tid & 63) == 0 && j < hidden && v > 0.0f) atomicMax(&amax[j], __float_as_uint(v));
    }
}

// One block per weight matrix W_j: max |element|.
__global__ __launch_bounds__(256) void calib_weight_kernel(const float* __restrict__ W, int din, unsigned* amax_w) {
    const int j = blockIdx.x;
    const int64_t off = j == 0 ? 0 : (int64_t)kWidth * din + (int64_t)(j - 1) * kWidth * kWidth;
    const int64_t cnt = j == 0 ? (int64_t)kWidth * din : (int64_t)kWidth * kWidth;
    float m = 0.0f;
    for (int64_t e = threadIdx.x; e < cnt; e += blockDim.x) m = fmaxf(m, fabsf(W[off + e]));
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    __shared__ float part[4];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) amax_w[j] = __float_as_uint(fmaxf(fmaxf(part[0], part[1]), fmaxf(part[2], part[3])));
}

size_t calib_workspace_bytes(int64_t n, int din) {
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    return al((size_t)n * din * 4) + al((size_t)n * 4) + 256;
}

hipError_t launch_calibrate(const FwdArgs& enc, int levels, int grid_dtype, int num_cus, int32_t mlp, const float* W,
                            int din, int hidden, void* ws, unsigned* amax_host, hipStream_t s) {
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const int64_t n = enc.n;
    uint8_t* p = reinterpret_cast<uint8_t*>(ws);
    unsigned* amax = reinterpret_cast<unsigned*>(p + al((size_t)n * din * 4) + al((size_t)n * 4));
    hipLaunchKernelGGL(calib_zero_kernel, dim3(1), dim3(64), 0, s, amax, 2 * kMaxHidden);
    if (n > 0) {
        FwdArgs a = enc;
        a.features = reinterpret_cast<float*>(p);
        a.status_out = reinterpret_cast<int32_t*>(p + al((size_t)n * din * 4));
        hipError_t e = launch_encode(levels, grid_dtype, a, num_cus, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(calib_act_kernel, dim3((unsigned)((n + kCalibBlock - 1) / kCalibBlock)), dim3(kCalibBlock), 0, s, a.features,
                           a.status_out, a.ids, a.objs, mlp, n, W, din, hidden, amax);
    }
    hipLaunchKernelGGL(calib_weight_kernel, dim3((unsigned)hidden), dim3(256), 0, s, W, din, amax + kMaxHidden);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(amax_host, amax, sizeof(unsigned) * 2 * kMaxHidden, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
}

}  // namespace nif
