// Hand-written gfx950 kernels that do not depend on the diagram graph:
//   dmc_sample_kernel   Philox4x32-10 -> VEGAS map -> physical map (HBM-write bound)
//   dmc_fold_kernel     fixed-order FP64 fold of per-block partial sums
//   dmc_hist_*          VEGAS importance histogram, integer (order-independent) accumulation
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace dmc {

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 multiplies.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

constexpr int kMaxDim = 4 * 6 - 1;

// One thread per sample; the order is a template parameter so that the coordinates stay in
// registers.
template <int N>
__global__ void __launch_bounds__(256) dmc_sample_kernel(SampleArgs a) {
    constexpr int D = 4 * N - 1;
    __shared__ float edges[kMaxDim * 129];
    const int ne = D * (a.n_bins + 1);
    if (a.kind == 1)
        for (int i = threadIdx.x; i < ne; i += blockDim.x) edges[i] = a.edges[i];
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < a.n; s += stride) {
        const uint64_t idx = a.first + (uint64_t)s;
        float y[D];
        float J = 1.0f;
#pragma unroll
        for (int b4 = 0; b4 * 4 < D; ++b4) {
            uint32_t c[4] = {(uint32_t)idx, (uint32_t)(idx >> 32), (uint32_t)b4, 0u};
            philox4x32_10(c, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const int d = b4 * 4 + w;
                if (d < D) {
                    const uint32_t m = c[w] >> 8;
                    if (a.kind == 1) {
                        // bin and fraction from the integer (2m + 1) B / 2^25: exact bin choice
                        const uint32_t t = (2u * m + 1u) * (uint32_t)a.n_bins;
                        const int bin = (int)(t >> 25);
                        const float fr = (float)(t & 0x1FFFFFFu) * 0x1p-25f;
                        const float lo = edges[d * (a.n_bins + 1) + bin];
                        const float hi = edges[d * (a.n_bins + 1) + bin + 1];
                        y[d] = __builtin_fmaf(fr, hi - lo, lo);
                        J *= (float)a.n_bins * (hi - lo);
                    } else {
                        y[d] = ((float)m + 0.5f) * 0x1p-24f;
                    }
                }
            }
        }
        // physical map: ball |q| <= R in spherical coordinates, times in [0, beta)
#pragma unroll
        for (int l = 0; l < N; ++l) {
            const float r = a.qmax * y[3 * l];
            const float ct = __builtin_fmaf(2.0f, y[3 * l + 1], -1.0f);
            const float st = __builtin_sqrtf(__builtin_fmaxf(0.0f, __builtin_fmaf(-ct, ct, 1.0f)));
            float sp, cp;
            sincospif(2.0f * y[3 * l + 2], &sp, &cp);
            a.x[(int64_t)(3 * l) * a.ld + s] = r * st * cp;
            a.x[(int64_t)(3 * l + 1) * a.ld + s] = r * st * sp;
            a.x[(int64_t)(3 * l + 2) * a.ld + s] = r * ct;
            J *= a.jl * r * r;
        }
#pragma unroll
        for (int j = 1; j < N; ++j) a.x[(int64_t)(3 * N + j - 1) * a.ld + s] = a.beta * y[3 * N + j - 1];
        a.jac[s] = J * a.jt;
    }
}

// totals[i] += sum_b partial[b][i] in a fixed order: thread t takes b = t, t + 256, ...;
// then a fixed LDS tree.  Block i handles entry i; the extra last block folds the counters.
__global__ void __launch_bounds__(256) dmc_fold_kernel(const double* partial, int nb, int st2, double* totals,
                                                      const unsigned int* nonfin_part,
                                                      unsigned long long* nonfin_tot) {
    __shared__ double red[256];
    const int i = blockIdx.x;
    double v = 0.0;
    if (i < st2) {
        for (int b = threadIdx.x; b < nb; b += 256) v += partial[(int64_t)b * st2 + i];
    } else {
        for (int b = threadIdx.x; b < nb; b += 256) v += (double)nonfin_part[b];
    }
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (i < st2)
            totals[i] += red[0];
        else
            *nonfin_tot += (unsigned long long)red[0];
    }
}

__global__ void dmc_zero_u32_kernel(unsigned int* p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// pass 1: largest importance (non-negative floats order like their bit patterns)
__global__ void __launch_bounds__(256) dmc_hist_max_kernel(const float* imp, int64_t n, unsigned int* maxbits) {
    unsigned int m = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += stride) {
        const float v = imp[s];
        if (v > 0.0f && __builtin_isfinite(v)) m = max(m, __float_as_uint(v));
    }
    for (int o = 32; o > 0; o >>= 1) m = max(m, (unsigned int)__shfl_xor((int)m, o));
    __shared__ unsigned int wmax[4];
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) atomicMax(maxbits, max(max(wmax[0], wmax[1]), max(wmax[2], wmax[3])));
}

__device__ __forceinline__ double hist_scale(unsigned int maxbits, int64_t n) {
    // fixed point: n * max^2 * scale < 2^62, so 64-bit sums cannot overflow
    const double mx = (double)__uint_as_float(maxbits);
    const double top = mx * mx * (double)n;
    int e;
    frexp(top, &e);
    return ldexp(1.0, 62 - e);
}

// pass 2: per-sample imp^2 in fixed point into (dimension, bin) cells; integer adds commute,
// so the result does not depend on the order in which samples arrive.
__global__ void __launch_bounds__(256) dmc_hist_acc_kernel(HistArgs a) {
    __shared__ unsigned long long h[kMaxDim * 128];
    const int nc = a.dim * a.n_bins;
    for (int i = threadIdx.x; i < nc; i += blockDim.x) h[i] = 0ull;
    __syncthreads();
    if (*a.maxbits != 0u) {
        const double sc = hist_scale(*a.maxbits, a.n);
        const int64_t stride = (int64_t)gridDim.x * blockDim.x;
        for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < a.n; s += stride) {
            const float v = a.imp[s];
            if (!(v > 0.0f) || !__builtin_isfinite(v)) continue;
            const double dv = (double)v;
            const unsigned long long q = (unsigned long long)(dv * dv * sc);
            if (q == 0ull) continue;
            const uint64_t idx = a.first + (uint64_t)s;
            for (int b4 = 0; b4 * 4 < a.dim; ++b4) {
                uint32_t c[4] = {(uint32_t)idx, (uint32_t)(idx >> 32), (uint32_t)b4, 0u};
                philox4x32_10(c, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
                for (int w = 0; w < 4; ++w) {
                    const int d = b4 * 4 + w;
                    if (d >= a.dim) break;
                    const uint32_t t = (2u * (c[w] >> 8) + 1u) * (uint32_t)a.n_bins;
                    atomicAdd(&h[d * a.n_bins + (int)(t >> 25)], q);
                }
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nc; i += blockDim.x)
        if (h[i]) atomicAdd(&a.hist_u64[i], h[i]);
}

// pass 3: convert to FP64 and add to the running histogram; clear the integer cells
__global__ void dmc_hist_fin_kernel(unsigned long long* hu, double* hd, int nc, const unsigned int* maxbits,
                                    int64_t n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nc) return;
    if (*maxbits != 0u) hd[i] += (double)hu[i] / hist_scale(*maxbits, n);
    hu[i] = 0ull;
}

// ---- launch wrappers ----
hipError_t launch_sample(const SampleArgs& a, int n_cu, hipStream_t st) {
    const int64_t want = (a.n + 255) / 256;
    const int grid = (int)(want < (int64_t)n_cu * 16 ? want : (int64_t)n_cu * 16);
    if (grid <= 0) return hipSuccess;
    switch (a.order) {
        case 1: hipLaunchKernelGGL(dmc_sample_kernel<1>, dim3(grid), dim3(256), 0, st, a); break;
        case 2: hipLaunchKernelGGL(dmc_sample_kernel<2>, dim3(grid), dim3(256), 0, st, a); break;
        case 3: hipLaunchKernelGGL(dmc_sample_kernel<3>, dim3(grid), dim3(256), 0, st, a); break;
        case 4: hipLaunchKernelGGL(dmc_sample_kernel<4>, dim3(grid), dim3(256), 0, st, a); break;
        case 5: hipLaunchKernelGGL(dmc_sample_kernel<5>, dim3(grid), dim3(256), 0, st, a); break;
        case 6: hipLaunchKernelGGL(dmc_sample_kernel<6>, dim3(grid), dim3(256), 0, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Block partials of the allocation-free evaluation (dmc_eval_accumulate_noalloc): FP64 partial sums and
// non-finite counts.  Host code reaches it only through scratch_address.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_address(void** out) { return hipGetSymbolAddress(out, HIP_SYMBOL(scratch)); }

hipError_t launch_fold(const double* partial, int nb, int st2, double* totals, const unsigned int* nonfin_part,
                       unsigned long long* nonfin_tot, hipStream_t st) {
    hipLaunchKernelGGL(dmc_fold_kernel, dim3(st2 + 1), dim3(256), 0, st, partial, nb, st2, totals, nonfin_part,
                       nonfin_tot);
    return hipGetLastError();
}

hipError_t launch_hist(const HistArgs& a, int n_cu, hipStream_t st) {
    hipLaunchKernelGGL(dmc_zero_u32_kernel, dim3(1), dim3(64), 0, st, a.maxbits, 1);
    const int64_t want = (a.n + 255) / 256;
    const int grid = (int)(want < (int64_t)n_cu * 8 ? want : (int64_t)n_cu * 8);
    if (grid <= 0) return hipGetLastError();
    hipLaunchKernelGGL(dmc_hist_max_kernel, dim3(grid), dim3(256), 0, st, a.imp, a.n, a.maxbits);
    hipLaunchKernelGGL(dmc_hist_acc_kernel, dim3(grid), dim3(256), 0, st, a);
    const int nc = a.dim * a.n_bins;
    hipLaunchKernelGGL(dmc_hist_fin_kernel, dim3((nc + 255) / 256), dim3(256), 0, st, a.hist_u64, a.hist, nc,
                       a.maxbits, a.n);
    return hipGetLastError();
}

}  // namespace dmc
