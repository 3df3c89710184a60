// Device-rate probes, for putting the walk's roofline fraction beside the rates
// this build can reach: the vector ALU's FP32 FMA rate as the walk kernels are
// compiled (one FMA per lane and instruction: the packed two-wide forms are
// switched off), and the BF16 matrix cores' rate on the walk's MFMA shape.
#include "ggns_common.h"

namespace ggns {
namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeChains = 8;   // independent FMA chains per thread
constexpr int kProbeAcc = 4;      // independent MFMA accumulators per wavefront

typedef __bf16 probe_bf16x8 __attribute__((ext_vector_type(8)));
typedef float probe_floatx4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(kProbeThreads)
valu_probe_kernel(float a, float b, int iters, float *out) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float v[kProbeChains];
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) v[k] = (float)(threadIdx.x & 63) * 0.015625f + (float)k;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kProbeChains; ++k) v[k] = __builtin_fmaf(v[k], a, b);
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) s += v[k];
    out[gid] = s;
}

__global__ void __launch_bounds__(kProbeThreads)
mfma_probe_kernel(float a, float b, int iters, float *out) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const __bf16 ab = (__bf16)a, bb = (__bf16)b;
    const probe_bf16x8 A = {ab, ab, ab, ab, ab, ab, ab, ab};
    const probe_bf16x8 B = {bb, bb, bb, bb, bb, bb, bb, bb};
    probe_floatx4 c[kProbeAcc];
#pragma unroll
    for (int k = 0; k < kProbeAcc; ++k) c[k] = probe_floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kProbeAcc; ++k)
            c[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B, c[k], 0, 0, 0);
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < kProbeAcc; ++k) s += (c[k][0] + c[k][1]) + (c[k][2] + c[k][3]);
    out[gid] = s;
}

bool probe_args_ok(int32_t blocks, int32_t iters, const float *out) {
    return blocks >= 1 && blocks <= (1 << 20) && iters >= 0 && out != nullptr;
}

}  // namespace
}  // namespace ggns

using namespace ggns;

int ggns_probe_valu(int32_t blocks, int32_t iters, float a, float b, float *out_dev, void *stream) {
    if (!probe_args_ok(blocks, iters, out_dev)) return GGNS_EINVAL;
    hipLaunchKernelGGL(valu_probe_kernel, dim3(blocks), dim3(kProbeThreads), 0,
                       reinterpret_cast<hipStream_t>(stream), a, b, iters, out_dev);
    return hipGetLastError() == hipSuccess ? GGNS_OK : GGNS_EHIP;
}

int ggns_probe_mfma(int32_t blocks, int32_t iters, float a, float b, float *out_dev, void *stream) {
    if (!probe_args_ok(blocks, iters, out_dev)) return GGNS_EINVAL;
    hipLaunchKernelGGL(mfma_probe_kernel, dim3(blocks), dim3(kProbeThreads), 0,
                       reinterpret_cast<hipStream_t>(stream), a, b, iters, out_dev);
    return hipGetLastError() == hipSuccess ? GGNS_OK : GGNS_EHIP;
}
