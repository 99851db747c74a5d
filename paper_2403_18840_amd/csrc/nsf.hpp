// Neural spline flow (Appendix A): rational-quadratic spline couplings with NSF_K bins on [0, 1], a
// residual conditioner with two hidden layers of NSF_H ReLU units, uniform base.  Parameters are one
// FP32 vector, per layer W1 [H][dA], b1 [H], W2 [H][H], b2 [H], W3 [P][H], b3 [P] (P = NSF_NP dB),
// row-major, layers in application order.  Spline parameters of transformed coordinate j: theta[j NP ..]
// = K width logits, K height logits, K - 1 interior derivative logits; widths and heights
// m + (1 - K m) softmax, interior derivatives m + softplus, boundary derivatives 1, m = 1e-3.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dmc {

constexpr int NSF_K = 8;
constexpr int NSF_H = 32;
constexpr int NSF_NP = 3 * NSF_K - 1;
constexpr int NSF_MAXD = 23;

struct NsfArgs {
    const float* params;
    const int* offs;   // [L]: float offset of each layer's parameters
    const int* aidx;   // [L][NSF_MAXD]: kept coordinates
    const int* bidx;   // [L][NSF_MAXD]: transformed coordinates
    const int* dA;     // [L]
    int n_layers, dim;
    // points: u_in [D][ld], or (u_in == NULL) the Philox uniforms (seed, first + i) of the uniform sampler
    const float* u_in;
    uint64_t seed, first;
    int64_t n, ld;
    // outputs
    float* x;        // [D][ld] (sampling)
    float* jac;      // [n] (sampling)
    float* u_out;    // nullable [D][ld]
    float* lq_out;   // nullable [n]: log q(u')
    float* jv_out;   // nullable [n]: the grid's Jacobian at u' (inverse pass)
    float* zs;       // nullable [L + 1][D][n]: z_l of the inverse pass, l = L .. 0 (training)
    // base points of the flow for the random walk in its base space, [D][ld_z]: given (sampling, replacing the
    // Philox draws) or returned (inverse pass); nullable
    const float* z_in;
    float* z0_out;
    int64_t ld_z;
    float* jf_out;   // nullable [n]: the flow's own weight J_phys J_V J_t / q_flow at the point (sampling; inverse
                     // pass with a sampler's grid)
    // grid and physical map (sampling; jv_out)
    const float* edges;
    int n_bins;
    float beta, qmax, jl, jt;
    float mix_f, mix_g, mix_u;
};

// flow share of the mixture: Philox z -> couplings -> u' -> VEGAS map -> physical map, weight vs the mixture
hipError_t launch_nsf_sample(const NsfArgs& a, int n_cu, hipStream_t st);
// u' -> log q(u') by the inverse couplings (optionally J_V(u'), u' itself when drawn, and every z_l)
hipError_t launch_nsf_inverse(const NsfArgs& a, int n_cu, hipStream_t st);

// base-space random walk: z <- z + sigma xi wrapped onto [0, 1), xi standard normals from Philox
hipError_t launch_nsf_walk(float* z, int D, int64_t n, int64_t ld, float sigma, uint64_t seed, uint64_t first,
                           int n_cu, hipStream_t st);

// Reverse sweep of one layer of the weighted forward KL L = -sum_i w_i log q(u_i) / sum_i w_i.
struct NsfBackArgs {
    const float* params;
    int off, dA, dB, dim;
    const int* aidx;   // this layer's kept coordinates (device)
    const int* bidx;   // this layer's transformed coordinates (device)
    const float* z;    // [D][n]: z_l, the layer's output (input of its inverse)
    float* adj;        // [D][n]: in: dL/dz_{l-1}; out: dL/dz_l
    const float* w;    // [n]
    const double* inv_wsum;
    int64_t n;
    // per-sample vectors for the weight gradients, [rows][n]
    float* d_theta;    // [P][n]
    float* a2;         // [H][n]
    float* d_pre2;     // [H][n]
    float* a1;         // [H][n]
    float* d_pre1;     // [H][n]
    float* zA;         // [dA][n]
};
hipError_t launch_nsf_backward(const NsfBackArgs& a, int n_cu, hipStream_t st);

// out_partial[c][i][j] = sum over the samples of chunk c of A[i][n] B[j][n] (j < rowsB <= 32), and
// out_partial[c][i][rowsB] = sum of A[i][n] (the bias gradient); FP32 matrix cores, deterministic order
int nsf_outer_chunks(int64_t n);
hipError_t launch_nsf_outer(const float* A, int rowsA, const float* B, int rowsB, int64_t n, float* partial,
                            hipStream_t st);
// grad = the weights [rowsA][rowsB] then the biases [rowsA]: the sum over chunks of partial, in a fixed order
hipError_t launch_nsf_outer_fold(const float* partial, int rowsA, int rowsB, int64_t n, float* grad, hipStream_t st);
// the loss sums: per block (sum w, sum w lq) in FP64
hipError_t launch_nsf_loss(const float* w, const float* lq, int64_t n, double* partial, int nblk, hipStream_t st);
// Adam on the FP32 parameters (beta1 0.9, beta2 0.999, eps 1e-8); non-finite gradients are skipped
hipError_t launch_nsf_adam(float* params, float* m, float* v, const float* grad, int64_t count, int64_t step,
                           float lr, hipStream_t st);

}  // namespace dmc
