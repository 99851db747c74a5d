// Argument blocks and launchers of the graph-independent kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dmc {

struct SampleArgs {
    uint64_t seed, first;
    int64_t n, ld;
    float* x;
    float* jac;
    const float* edges;  // device [dim][n_bins + 1] (VEGAS only)
    int kind, order, dim, n_bins;
    float beta, qmax;
    float jl;  // 4 pi R: per-loop Jacobian factor (times r^2)
    float jt;  // beta^(n-1): Jacobian of the times
};

struct HistArgs {
    const float* imp;
    int64_t n;
    uint64_t seed, first;
    int dim, n_bins;
    unsigned int* maxbits;         // device scratch, 1 word
    unsigned long long* hist_u64;  // device [dim][n_bins], zero on entry
    double* hist;                  // device [dim][n_bins], running FP64 histogram
};

hipError_t launch_sample(const SampleArgs& a, int n_cu, hipStream_t st);
hipError_t launch_fold(const double* partial, int nb, int st2, double* totals, const unsigned int* nonfin_part,
                       unsigned long long* nonfin_tot, hipStream_t st);
hipError_t launch_hist(const HistArgs& a, int n_cu, hipStream_t st);

// The allocation-free evaluation's block partials live in a static device array of this size (each GPU
// holds its own copy until the process ends); scratch_address gives the current device's copy.
constexpr size_t kScratchBytes = 4u << 20;
hipError_t scratch_address(void** out);

}  // namespace dmc
