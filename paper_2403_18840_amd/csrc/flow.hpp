// Layouts and launchers of the affine-coupling flow kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dmc {

constexpr int FH = 128;    // hidden width
constexpr int FKIN = 16;   // first-layer input width: z_A (<= 12), the bias input, zero padding
constexpr int FNOUT = 32;  // last-layer outputs: s_hat in 0..15, t in 16..31
constexpr int ZMAX = 24;   // largest dimension + 1
constexpr float FLOW_SMAX = 2.0f;

// FP32 master parameters of one layer (the flat order of dmc_flow_set_params)
constexpr int OFF_W1T = 0;                       // [128][16]; column d_A is the first-layer bias
constexpr int OFF_W2T = OFF_W1T + FH * FKIN;     // [128][128]
constexpr int OFF_B2 = OFF_W2T + FH * FH;        // [128]
constexpr int OFF_W3T = OFF_B2 + FH;             // [32][128]
constexpr int OFF_B3 = OFF_W3T + FNOUT * FH;     // [32]
constexpr int LAYER_SIZE = OFF_B3 + FNOUT;       // 22688

// BF16 shadow of one layer: forward operands (rows = outputs) and backward operands (rows = inputs)
constexpr int SH_W1T = 0;                        // [128][16]
constexpr int SH_W2T = SH_W1T + FH * FKIN;       // [128][128]
constexpr int SH_W3T = SH_W2T + FH * FH;         // [32][128]
constexpr int SH_W1 = SH_W3T + FNOUT * FH;       // [32][128]: rows 0..15 = W1t^T, rows 16..31 zero
constexpr int SH_W2 = SH_W1 + 32 * FH;           // [128][128] = W2t^T
constexpr int SH_W3 = SH_W2 + FH * FH;           // [128][32] = W3t^T
// Forward weights in MFMA fragment order (44 fragments of 64 lanes x 8 BF16; fragment f, lane l,
// element t at SH_FRAG + 512 f + 8 l + t): the A operands of the 32x32x16 products, laid out so
// that the ReLU'd accumulator registers of one layer are the B operands of the next.
//   f = ot (0..3):            W1t[32 ot + l%32][8 (l/32) + t]
//   f = 4 + 8 ot + sg:        W2t[32 ot + l%32][rho(sg, l/32, t)]
//   f = 36 + sg:              W3t[l%32][rho(sg, l/32, t)]
// with rho(sg, h, t) = 32 (sg/2) + 16 (sg%2) + 8 (t/4) + 4 h + t%4, the hidden unit that the
// accumulator register 8 (sg%2) + t of output tile sg/2 holds in lane half h.
constexpr int NFRAG = 44;
constexpr int SH_FRAG = SH_W3 + FH * FNOUT;
// the FP32 biases b2 [128] and b3 [32] as raw words right after the fragments (1 KiB with padding):
// fragments and biases of a layer form 45 contiguous 1 KiB chunks
constexpr int SH_BIAS = SH_FRAG + NFRAG * 512;
constexpr int NCHUNK = NFRAG + 1;
constexpr int SHADOW_LAYER = SH_BIAS + 512;

// slot of hidden input c within a fragment row: (sg, h, t) with rho(sg, h, t) = c
__device__ __forceinline__ int frag_slot(int sg_base, int row, int c) {
    const int sg = 2 * (c >> 5) + ((c & 31) >> 4);
    const int h = (c & 7) >> 2;
    const int t = 4 * ((c & 15) >> 3) + (c & 3);
    return SH_FRAG + (sg_base + sg) * 512 + (32 * h + row) * 8 + t;
}

// BF16 of an FP32 master by round-to-nearest-even on its bit pattern.  The shadow must be a function of the
// stored FP32 value alone: a plain conversion lets the compiler fuse it with the FP64 -> FP32 rounding of
// the Adam update into one correctly rounded FP64 -> BF16 conversion, which differs from rounding the
// stored master at BF16 ties, so a shadow rebuilt from the masters (set_params, checkpoint load) would
// not equal the one Adam wrote.  Masters are finite (set_params refuses others, Adam skips non-finite
// gradients).
__device__ __forceinline__ __bf16 master_to_bf16(float th) {
    unsigned u = __builtin_bit_cast(unsigned, th);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return __builtin_bit_cast(__bf16, (unsigned short)(u >> 16));
}

__device__ __forceinline__ void write_shadow(__bf16* shadow, int l, int q, float th) {
    __bf16* s = shadow + (size_t)l * SHADOW_LAYER;
    const __bf16 b = master_to_bf16(th);
    if (q < OFF_W2T) {
        const int r = q / FKIN, k = q % FKIN;
        s[SH_W1T + r * FKIN + k] = b;
        s[SH_W1 + k * FH + r] = b;
        s[SH_FRAG + (r >> 5) * 512 + (32 * (k >> 3) + (r & 31)) * 8 + (k & 7)] = b;
    } else if (q < OFF_B2) {
        const int o = (q - OFF_W2T) / FH, i = (q - OFF_W2T) % FH;
        s[SH_W2T + o * FH + i] = b;
        s[SH_W2 + i * FH + o] = b;
        s[frag_slot(4 + 8 * (o >> 5), o & 31, i)] = b;
    } else if (q >= OFF_W3T && q < OFF_B3) {
        const int o = (q - OFF_W3T) / FH, i = (q - OFF_W3T) % FH;
        s[SH_W3T + o * FH + i] = b;
        s[SH_W3 + i * FNOUT + o] = b;
        s[frag_slot(36, o, i)] = b;
    } else if (q < OFF_W3T) {
        ((float*)(s + SH_BIAS))[q - OFF_B2] = th;
    } else {
        ((float*)(s + SH_BIAS))[FH + q - OFF_B3] = th;
    }
}

struct FlowSampleArgs {
    uint64_t seed, first;
    int64_t n, ld;
    float* x;
    float* jac;
    float* u_out;   // nullable [D][ld]: the flow output u' (VEGAS coordinates)
    float* lq_out;  // nullable [n]: log q(u')
    const float* edges;
    const float* master;
    const __bf16* shadow;
    const int* aidx;  // [L][16]
    const int* bidx;  // [L][16]
    const int* dA;    // [L]
    int n_layers, n_bins;
    float beta, qmax, jl, jt;
    // shares of the sampling mixture a_f q_flow + a_g (grid) + a_u (uniform): the weight of a point is
    // J_phys J_V / (a_f q_flow(u') + a_g + a_u J_V), J_V the grid's Jacobian at u'
    float mix_f, mix_g, mix_u;
};

// The uniform share of the mixture: y = Philox uniforms (as the uniform sampler draws them),
// physical map, and the grid coordinates u' = G^-1(y) with the grid's Jacobian J_V(u').
struct FlowUniformArgs {
    uint64_t seed, first;
    int64_t n, ld, ldu;
    float* x;        // [D][ld]
    float* jac;      // [n]: J_phys
    float* u_out;    // [D][ldu]: u'
    float* jv_out;   // [n]: J_V(u')
    const float* edges;
    int n_bins, dim;
    float beta, qmax, jl, jt;
};

struct FlowTrainArgs {
    const float* u_in;  // nullable [D][ld]: training points u'; NULL = Philox uniforms (seed, first)
    uint64_t seed, first;
    int64_t n, ld;
    int64_t lda;        // row stride of the activation buffers: n rounded up to a multiple of 16
    const float* w;     // [n] importance weights
    const double* inv_wsum;  // device: 1 / sum(w) (the weights enter normalised)
    const float* master;
    const __bf16* shadow;
    const int* aidx;
    const int* bidx;
    const int* dA;
    int n_layers, dim;
    float* states;      // [L][D][n]
    float* G;           // [D][n]
    float* weff;        // [n]: w / sum(w), or 0 for a sample whose density is not finite
    float* lq_out;      // nullable [n]
    float* u_out;       // nullable [D][ld]: the points u' used (Philox uniforms when u_in is NULL)
    const float* edges; // with jv_out: the VEGAS grid [D][n_bins + 1]
    int n_bins;
    float* jv_out;      // nullable [n]: J_V at the Philox points (bin by the sampler's integer rule)
    float* loss_part;   // [blocks]
    __bf16* act_x1;     // [16][n]
    __bf16* act_h1;     // [128][n]
    __bf16* act_h2;     // [128][n]
    __bf16* act_do;     // [32][n]
    __bf16* act_dp2;    // [128][n]
    __bf16* act_dp1;    // [128][n]
};

struct FlowAdamArgs {
    const float* partial;  // [L][nblk_max][LAYER_SIZE]
    int nblk, nblk_max, n_layers, apply;
    float* master;
    float* m;
    float* v;
    __bf16* shadow;
    float* grad_out;       // nullable [P]
    double lr, b1, b2, eps, b1t, b2t;  // b1t = b1^step, b2t = b2^step
};

int flow_sample_lds_bytes(int dim);
hipError_t launch_flow_sample(const FlowSampleArgs& a, int dim, int n_cu, hipStream_t st);
int flow_train_blocks(int64_t n, int n_cu);    // grid of the backward sweep (128 samples per block pass)
int flow_inverse_blocks(int64_t n, int n_cu);  // grid of the inverse pass (one 512-thread block per CU at most)
hipError_t launch_flow_inverse(const FlowTrainArgs& a, int nblk, hipStream_t st);
hipError_t launch_flow_backward(const FlowTrainArgs& a, int nblk, int layer, int wg_chunk, int wg_blocks,
                                float* partial_layer, hipStream_t st);
hipError_t launch_flow_sums(const float* w, int64_t n, double* out, hipStream_t st);
hipError_t launch_flow_loss(const float* loss_part, int nblk, double* out, hipStream_t st);
hipError_t launch_flow_adam(const FlowAdamArgs& a, int n_cu, hipStream_t st);
// jac[i] <- jac[i] (jv[i] if scale_jv) / (a_f exp(lq[i]) + a_g + a_u jv[i])
hipError_t launch_flow_mix(float* jac, const float* lq, const float* jv, int64_t n, float a_f, float a_g, float a_u,
                           bool scale_jv, hipStream_t st);
hipError_t launch_flow_uniform(const FlowUniformArgs& a, int n_cu, hipStream_t st);
hipError_t launch_flow_shadow(const float* master, __bf16* shadow, int n_layers, int n_cu, hipStream_t st);

}  // namespace dmc
