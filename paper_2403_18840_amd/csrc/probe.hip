// Throughput probes that check the roofline denominators on the device at hand: FP32 fused multiply-add
// (unpacked), the hardware 2^x and reciprocal, and a device-to-device copy through HBM.  Each lane runs
// eight independent chains so that issue, not latency, limits the loop; the results are stored so that the
// compiler keeps the work.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "probe.hpp"

namespace dmc {

constexpr int CHAINS = 8;

__global__ void __launch_bounds__(256) dmc_probe_fma_kernel(float* out, int iters, float b, float c) {
    float a[CHAINS];
#pragma unroll
    for (int i = 0; i < CHAINS; ++i) a[i] = (float)(threadIdx.x + i);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int r = 0; r < 16; ++r)
#pragma unroll
            for (int i = 0; i < CHAINS; ++i) a[i] = __builtin_fmaf(a[i], b, c);
    }
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < CHAINS; ++i) s += a[i];
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// kind 1: v <- 2^-v (v_exp_f32 with its input negation folded); kind 2: v <- 1 / v (v_rcp_f32)
template <int Kind>
__global__ void __launch_bounds__(256) dmc_probe_trans_kernel(float* out, int iters) {
    float a[CHAINS];
#pragma unroll
    for (int i = 0; i < CHAINS; ++i) a[i] = 0.5f + 0.01f * (float)(threadIdx.x % 7 + i);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int r = 0; r < 16; ++r)
#pragma unroll
            for (int i = 0; i < CHAINS; ++i)
                a[i] = Kind == 1 ? __builtin_amdgcn_exp2f(-a[i]) : __builtin_amdgcn_rcpf(a[i]);
    }
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < CHAINS; ++i) s += a[i];
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) dmc_probe_copy_kernel(const float4* in, float4* out, int64_t n4) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = in[i];
}

hipError_t launch_probe(int kind, float* out, int blocks, int iters, const float* in, float* dst, int64_t n4,
                        hipStream_t st) {
    switch (kind) {
        case 0:
            hipLaunchKernelGGL(dmc_probe_fma_kernel, dim3(blocks), dim3(256), 0, st, out, iters, 0.999f, 1e-3f);
            break;
        case 1:
            hipLaunchKernelGGL(dmc_probe_trans_kernel<1>, dim3(blocks), dim3(256), 0, st, out, iters);
            break;
        case 2:
            hipLaunchKernelGGL(dmc_probe_trans_kernel<2>, dim3(blocks), dim3(256), 0, st, out, iters);
            break;
        case 3:
            hipLaunchKernelGGL(dmc_probe_copy_kernel, dim3(blocks), dim3(256), 0, st,
                               reinterpret_cast<const float4*>(in), reinterpret_cast<float4*>(dst), n4);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace dmc
