// Affine-coupling normalizing flow on gfx950 BF16 MFMA (Appendix A: coupling layers, eq.
// coupling_layer; density by eq. NFtransform; forward-KL training).
//
// Network per coupling layer: X1 = [sigmoid(z_A), 1, 0..] (16) -> relu(X1 W1t^T) (128) -> relu(. W2t^T + b2)
// (128) -> . W3t^T + b3 (32): s = S_MAX tanh(O[b]), t = O[16 + b] for the d_B transformed dims.
// All matmuls run as v_mfma_f32_32x32x16_bf16 in the transposed form H^T = W^T X^T: the A operand
// is a weight tile (rows = outputs, 8 consecutive K per lane), the B operand an activation tile
// (K = features, columns = 32 samples), the FP32 result lane l holds column l%32 and rows
// 8g + 4(l/32) + c.  Activations round to BF16 at every matmul input; bias, ReLU, tanh, exp and
// the log-density stay FP32.
//
//   dmc_flow_sample_kernel   Philox u -> logit -> 8 couplings -> sigmoid -> VEGAS map -> physical
//                            map; x, J = J_phys J_VEGAS / q.  Weights of one layer staged in LDS
//                            and shared by the block's 256 samples (lane = sample).
//   dmc_flow_inverse_kernel  u' -> z_0 through the inverse couplings; stores every state and
//                            log q (density for training and for tests).
//   dmc_flow_bwd_kernel      one layer of the reverse sweep: recompute the network, back through
//                            the coupling and the network; writes the activations and their
//                            gradients for the weight-gradient products.
//   dmc_flow_wgrad_kernel    split-K weight gradients of one layer over samples (fixed order).
//   dmc_flow_adam_kernel     fixed-order fold of the partial gradients, Adam on the FP32 masters,
//                            BF16 shadows in forward and backward layouts.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "flow.hpp"

namespace dmc {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef short i16x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x16 mfma(bf16x8 a, bf16x8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void philox(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0, n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[1] = (uint32_t)p1;
        c[3] = (uint32_t)p0;
        c[0] = n0;
        c[2] = n2;
    }
}

// Hardware exp2 / log2 / reciprocal (about 1 ulp).  The flow uses them on both sides of every
// density (the map and its log-determinant share each computed s), so their rounding changes the
// density at the 1e-7 level only.
constexpr float LOG2E = 1.44269504088896341f, LN2 = 0.693147180559945309f;
__device__ __forceinline__ float fexp(float x) { return __builtin_amdgcn_exp2f(x * LOG2E); }
__device__ __forceinline__ float flog(float x) { return __builtin_amdgcn_logf(x) * LN2; }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fsigmoid(float z) { return frcp(1.0f + fexp(-z)); }
// tanh x = 1 - 2 / (1 + e^{2x}): saturates to +-1 without overflow; absolute error ~1e-7
__device__ __forceinline__ float ftanh(float x) { return 1.0f - 2.0f * frcp(1.0f + fexp(2.0f * x)); }

// log sigma'(z) = -|z| - 2 log(1 + e^{-|z|})
__device__ __forceinline__ float log_sig_prime(float z) {
    const float a = fabsf(z);
    return -a - 2.0f * flog(1.0f + fexp(-a));
}

// logit of the 24-bit uniform u = (m + 1/2) 2^-24, m = w >> 8: log(m + 1/2) - log(2^24 - 1 - m + 1/2).
// Both operands are exact in FP32 wherever their logarithm is sensitive to rounding (below 2^23),
// so the result is finite for every word (u itself rounds to 1 in FP32 at m = 2^24 - 1).
__device__ __forceinline__ float philox_logit(uint32_t w) {
    const uint32_t m = w >> 8;
    return flog((float)m + 0.5f) - flog((float)(0xFFFFFFu - m) + 0.5f);
}

// ---------------------------------------------------------------- LDS geometry
// Row strides padded by 8 BF16 (16 B) so that 16 lanes reading 16 B each hit distinct banks.
constexpr int XS = FKIN + 8;    // 24
constexpr int HS = FH + 8;      // 136
constexpr int OS = FNOUT + 4;   // 36 floats

// One coupling layer in LDS: the 44 weight fragments (lane-contiguous, so every fragment read is
// one linear 1 KiB sweep without bank conflicts) and the biases: the 45 chunks of the shadow.
struct LayerLds {
    static constexpr int frag = 0;                  // bf16 [44][64][8]
    static constexpr int b2 = NFRAG * 1024;         // f32 [128]
    static constexpr int b3 = b2 + FH * 4;          // f32 [32]
    static constexpr int bytes = NCHUNK * 1024;     // 46080
};

// The sampler and the inverse pass: 512-thread blocks (8 waves, two per SIMD), one per CU.
// Two layer buffers: while the waves multiply with layer l, the next layer streams from L2
// straight into the other buffer (global_load_lds, 1 KiB per wave instruction), so the only
// synchronisation per layer is one barrier.  Per wave: the coupling states of its 64 samples
// (two 32-sample tiles), rows of D + 2 floats (an odd stride for odd D spreads the lanes' rows
// over the banks).
constexpr int PASS_WAVES = 8;
constexpr int PASS_THREADS = 64 * PASS_WAVES;
template <int D>
struct PassLds {
    static constexpr int ZS = D + 2;
    static constexpr int buf0 = 0;
    static constexpr int buf1 = LayerLds::bytes;
    static constexpr int z = 2 * LayerLds::bytes;   // f32 [8 waves][64][ZS]
    static constexpr int bytes = z + PASS_WAVES * 64 * ZS * 4;
};

typedef __attribute__((address_space(3))) void* lds_ptr;

// Start copying layer l's 45 chunks into an LDS buffer: wave w copies chunks w, w + 8, ...
__device__ __forceinline__ void prefetch_layer(char* buf, const __bf16* shadow, int l) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const char* src = (const char*)(shadow + (size_t)l * SHADOW_LAYER + SH_FRAG);
    for (int c = wv; c < NCHUNK; c += PASS_WAVES)
        __builtin_amdgcn_global_load_lds((const void*)(src + c * 1024 + lane * 16), (lds_ptr)(buf + c * 1024), 16, 0, 0);
}

// every copy this wave started has landed in LDS (and all its other memory operations are done)
__device__ __forceinline__ void wait_copies() { __builtin_amdgcn_s_waitcnt(0); }

__device__ __forceinline__ bf16x8 lds_frag(const char* sm, int f, int lane) {
    return *(const bf16x8*)(sm + LayerLds::frag + f * 1024 + lane * 16);
}

// BF16 rounding and ReLU of accumulator registers 8p .. 8p + 7: the B operand of one K-slice.
// ReLU acts on the rounded values as a packed signed 16-bit max against 0 (a BF16 with the sign
// bit set is a negative 16-bit integer, and the non-negative ones order like integers), which
// equals rounding after the ReLU: RNE keeps the sign, and -0 becomes +0.
__device__ __forceinline__ unsigned relu_pair(float a, float b) {
    const bf16x2 v = __builtin_convertvector((f32x2){a, b}, bf16x2);  // one packed RNE conversion
    return __builtin_bit_cast(unsigned, __builtin_elementwise_max(__builtin_bit_cast(i16x2, v), (i16x2){}));
}
__device__ __forceinline__ bf16x8 relu_slice(const f32x16& c, int p) {
    const u32x4 r = {relu_pair(c[8 * p], c[8 * p + 1]), relu_pair(c[8 * p + 2], c[8 * p + 3]),
                     relu_pair(c[8 * p + 4], c[8 * p + 5]), relu_pair(c[8 * p + 6], c[8 * p + 7])};
    return __builtin_bit_cast(bf16x8, r);
}

// bias in accumulator layout: register 4g + q of lane l holds row 8g + 4(l/32) + q
__device__ __forceinline__ f32x16 bias_acc(const float* b, int h) {
    f32x16 c;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const f32x4 v = *(const f32x4*)(b + 8 * g + 4 * h);
#pragma unroll
        for (int q = 0; q < 4; ++q) c[4 * g + q] = v[q];
    }
    return c;
}

// The network of the staged layer for two 32-sample tiles, all activations in registers:
// x1[tile] (B operands, K = 16 inputs) -> o[tile] (s_hat in registers 0..7, t in 8..15; see
// coupling_b for the unit each register holds).  The code issues the products of one output
// tile before rounding the previous tile's results, so the rounding overlaps the matrix core.
__device__ __forceinline__ void mlp_regs(const char* sm, const bf16x8 (&x1)[2], f32x16 (&o)[2]) {
    const int lane = threadIdx.x & 63, h = lane >> 5;
    bf16x8 h1[8][2];
    {
        f32x16 c[2][2];
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) {
            const bf16x8 aw = lds_frag(sm, ot, lane);
            c[ot & 1][0] = mfma(aw, x1[0], (f32x16){});
            c[ot & 1][1] = mfma(aw, x1[1], (f32x16){});
            if (ot > 0)
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) {
                    h1[2 * ot - 2][nt] = relu_slice(c[(ot - 1) & 1][nt], 0);
                    h1[2 * ot - 1][nt] = relu_slice(c[(ot - 1) & 1][nt], 1);
                }
        }
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            h1[6][nt] = relu_slice(c[1][nt], 0);
            h1[7][nt] = relu_slice(c[1][nt], 1);
        }
    }
    bf16x8 h2[8][2];
    const float* b2 = (const float*)(sm + LayerLds::b2);
    {
        f32x16 acc[2][2];
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) {
            const f32x16 bias = bias_acc(b2 + 32 * ot, h);
            f32x16* a2 = acc[ot & 1];
            {
                const bf16x8 aw = lds_frag(sm, 4 + 8 * ot, lane);
                a2[0] = mfma(aw, h1[0][0], bias);
                a2[1] = mfma(aw, h1[0][1], bias);
            }
#pragma unroll
            for (int sg = 1; sg < 8; ++sg) {
                const bf16x8 aw = lds_frag(sm, 4 + 8 * ot + sg, lane);
                a2[0] = mfma(aw, h1[sg][0], a2[0]);
                a2[1] = mfma(aw, h1[sg][1], a2[1]);
                if (sg == 2 && ot > 0)
#pragma unroll
                    for (int nt = 0; nt < 2; ++nt) {
                        h2[2 * ot - 2][nt] = relu_slice(acc[(ot - 1) & 1][nt], 0);
                        h2[2 * ot - 1][nt] = relu_slice(acc[(ot - 1) & 1][nt], 1);
                    }
            }
        }
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            h2[6][nt] = relu_slice(acc[1][nt], 0);
            h2[7][nt] = relu_slice(acc[1][nt], 1);
        }
    }
    const f32x16 b3 = bias_acc((const float*)(sm + LayerLds::b3), h);
    {
        const bf16x8 aw = lds_frag(sm, 36, lane);
        o[0] = mfma(aw, h2[0][0], b3);
        o[1] = mfma(aw, h2[0][1], b3);
    }
#pragma unroll
    for (int sg = 1; sg < 8; ++sg) {
        const bf16x8 aw = lds_frag(sm, 36 + sg, lane);
        o[0] = mfma(aw, h2[sg][0], o[0]);
        o[1] = mfma(aw, h2[sg][1], o[1]);
    }
}

// transformed unit whose (s_hat, t) sit in output registers (r, r + 8) of a lane in half h
__device__ __forceinline__ int coupling_b(int r, int h) { return r < 4 ? 4 * h + r : 4 + 4 * h + r; }

// X1 of one tile as the B operand: lane half h supplies inputs 8h .. 8h + 7 of its sample.
// ia: the layer's conditioning list in global memory (uniform: read through the scalar cache).
__device__ __forceinline__ bf16x8 x1_operand(const float* zr, const int* ia, int dA, int h) {
    bf16x8 v;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int k = 8 * h + t;
        const int zi = h ? ia[8 + t] : ia[t];
        const float x = k < dA ? fsigmoid(zr[zi]) : (k == dA ? 1.0f : 0.0f);
        v[t] = (__bf16)x;
    }
    return v;
}

// transformed-list entry of output register r (r < 8) in lane half h (ib: the layer's list)
__device__ __forceinline__ int coupling_z(const int* ib, int r, int h) {
    return r < 4 ? (h ? ib[4 + r] : ib[r]) : (h ? ib[8 + r] : ib[4 + r]);
}

// One coupling layer for the wave's two tiles, with the layer's weights in buf: the network
// (registers only), then the affine update of the transformed units this lane half owns and
// its share of the log-determinant.  Forward: z_B <- z_B e^s + t; inverse: z_B <- (z_B - t) e^-s.
// With s = 2 tanh(x) = 2 - 4 r, r = 1 / (1 + e^{2x}): e^{+-s} = 2^{+-(2 - 4r) log2 e}.
template <int D, bool INVERSE>
__device__ __forceinline__ void coupling_layer(const char* buf, float* zw, const int* ia, const int* ib, int dA,
                                               float (&lqp)[2]) {
    constexpr int ZS = D + 2;
    const int lane = threadIdx.x & 63, h = lane >> 5, j = lane & 31;
    const int dB = D - dA;
    bf16x8 x1[2];
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) x1[nt] = x1_operand(zw + (32 * nt + j) * ZS, ia, dA, h);
    f32x16 o[2];
    mlp_regs(buf, x1, o);
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        float* zr = zw + (32 * nt + j) * ZS;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            if (coupling_b(r, h) < dB) {
                const float rr = frcp(1.0f + __builtin_amdgcn_exp2f(o[nt][r] * (2.0f * LOG2E)));
                const float sv = __builtin_fmaf(-2.0f * FLOW_SMAX, rr, FLOW_SMAX);
                const int zi = coupling_z(ib, r, h);
                if (INVERSE)
                    zr[zi] = (zr[zi] - o[nt][r + 8]) * __builtin_amdgcn_exp2f(-sv * LOG2E);
                else
                    zr[zi] = __builtin_fmaf(zr[zi], __builtin_amdgcn_exp2f(sv * LOG2E), o[nt][r + 8]);
                lqp[nt] -= sv;
            }
        }
    }
    wave_sync();
}

// Forward sampling.  A wave owns 64 samples (tiles 0 and 1 of 32; lanes l and l + 32 share
// sample l % 32 of a tile: during the layers half h computes the Philox blocks, inputs and
// transformed units of its share, and at the end half h finishes tile h's samples).
template <int D>
__global__ void __launch_bounds__(PASS_THREADS) __attribute__((amdgpu_waves_per_eu(2)))
dmc_flow_sample_kernel(FlowSampleArgs a) {
    extern __shared__ __attribute__((aligned(16))) char sm[];
    constexpr int ZS = PassLds<D>::ZS;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, h = lane >> 5, j = lane & 31;
    float* zw = (float*)(sm + PassLds<D>::z) + wv * 64 * ZS;
    constexpr int N = (D + 1) / 4;  // loop momenta
    const int64_t nbatch = (a.n + PASS_THREADS - 1) / PASS_THREADS;
    const int L = a.n_layers;
    int g = 0;  // layers done by this block: layer buffer g & 1
    prefetch_layer(sm + PassLds<D>::buf0, a.shadow, 0);
    for (int64_t bt = blockIdx.x; bt < nbatch; bt += gridDim.x) {
        const int64_t base = bt * PASS_THREADS + wv * 64;
        float lqp[2];
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const int64_t s = base + 32 * nt + j;
            const uint64_t idx = a.first + (uint64_t)(s < a.n ? s : 0);
            float* zr = zw + (32 * nt + j) * ZS;
            lqp[nt] = 0.0f;
#pragma unroll
            for (int b4 = 0; b4 * 4 < D; ++b4) {
                if ((b4 & 1) != h) continue;
                uint32_t c[4] = {(uint32_t)idx, (uint32_t)(idx >> 32), (uint32_t)b4, 0u};
                philox(c, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    const int d = 4 * b4 + w;
                    if (d < D) {
                        const float z = philox_logit(c[w]);
                        zr[d] = z;
                        lqp[nt] += log_sig_prime(z);
                    }
                }
            }
        }
        for (int l = 0; l < L; ++l, ++g) {
            wait_copies();
            __syncthreads();  // layer l is in buffer g & 1; every wave is done with the other buffer
            if (l + 1 < L || bt + gridDim.x < nbatch)
                prefetch_layer(sm + ((g + 1) & 1 ? PassLds<D>::buf1 : PassLds<D>::buf0), a.shadow, l + 1 < L ? l + 1 : 0);
            coupling_layer<D, false>(sm + (g & 1 ? PassLds<D>::buf1 : PassLds<D>::buf0), zw, a.aidx + l * 16,
                                     a.bidx + l * 16, a.dA[l], lqp);
        }
        // tile h's sample: its log q is this lane's share plus the other half's
        const int64_t s = base + 32 * h + j;
        float lq = lqp[h] + __shfl_xor(lqp[1 - h], 32);
        if (s < a.n) {
            const float* zr = zw + (32 * h + j) * ZS;
            // u' = sigmoid(z_K); VEGAS map with the bin taken in FP32; physical map
            float J = 1.0f, jv = 1.0f;
            float y[D];
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const float z = zr[d];
                lq -= log_sig_prime(z);
                const float up = fsigmoid(z);
                if (a.u_out) a.u_out[(int64_t)d * a.ld + s] = up;
                const float ub = up * (float)a.n_bins;
                // clamp before the conversion: a non-finite output must not index outside the grid
                const int bin = (int)fminf(fmaxf(ub, 0.0f), (float)(a.n_bins - 1));
                const float fr = ub - (float)bin;
                const float lo = a.edges[d * (a.n_bins + 1) + bin];
                const float hi = a.edges[d * (a.n_bins + 1) + bin + 1];
                y[d] = __builtin_fmaf(fr, hi - lo, lo);
                jv *= (float)a.n_bins * (hi - lo);
            }
#pragma unroll
            for (int q = 0; q < N; ++q) {
                const float r = a.qmax * y[3 * q];
                const float ct = __builtin_fmaf(2.0f, y[3 * q + 1], -1.0f);
                const float st = __builtin_sqrtf(__builtin_fmaxf(0.0f, __builtin_fmaf(-ct, ct, 1.0f)));
                float sp, cp;
                sincospif(2.0f * y[3 * q + 2], &sp, &cp);
                a.x[(int64_t)(3 * q) * a.ld + s] = r * st * cp;
                a.x[(int64_t)(3 * q + 1) * a.ld + s] = r * st * sp;
                a.x[(int64_t)(3 * q + 2) * a.ld + s] = r * ct;
                J *= a.jl * r * r;
            }
#pragma unroll
            for (int jt = 1; jt < N; ++jt) a.x[(int64_t)(3 * N + jt - 1) * a.ld + s] = a.beta * y[3 * N + jt - 1];
            // weight against the mixture density: within 1/a_g of the grid's own weight and within
            // 1/a_u of the uniform sampler's in the flow's tails
            a.jac[s] = J * jv * a.jt / __builtin_fmaf(a.mix_f, fexp(lq), __builtin_fmaf(a.mix_u, jv, a.mix_g));
            if (a.lq_out) a.lq_out[s] = lq;
        }
    }
    wait_copies();  // no copy into LDS outlives the block
}

// Inverse pass u' -> z_0, same geometry as the sampler.  Stores (when asked) every state
// states[l][d][n] = z^(l) (the output of inverse layer l), log q, the effective weights
// w / sum(w), G[d][n] = d(-w lq)/dz_0 and the block's partial loss.
template <int D>
__global__ void __launch_bounds__(PASS_THREADS) __attribute__((amdgpu_waves_per_eu(2)))
dmc_flow_inverse_kernel(FlowTrainArgs a) {
    extern __shared__ __attribute__((aligned(16))) char sm[];
    constexpr int ZS = PassLds<D>::ZS;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, h = lane >> 5, j = lane & 31;
    float* zw = (float*)(sm + PassLds<D>::z) + wv * 64 * ZS;
    float loss = 0.0f;
    const int64_t nbatch = (a.n + PASS_THREADS - 1) / PASS_THREADS;
    const int L = a.n_layers;
    int g = 0;
    prefetch_layer(sm + PassLds<D>::buf0, a.shadow, L - 1);
    for (int64_t bt = blockIdx.x; bt < nbatch; bt += gridDim.x) {
        const int64_t base = bt * PASS_THREADS + wv * 64;
        float lqp[2], jvp[2] = {1.0f, 1.0f};
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const int64_t s = base + 32 * nt + j;
            const bool valid = s < a.n;
            float* zr = zw + (32 * nt + j) * ZS;
            lqp[nt] = 0.0f;
            if (a.u_in) {
                for (int d = h; d < D; d += 2) {
                    float up = valid ? a.u_in[(int64_t)d * a.ld + s] : 0.5f;
                    // outputs that rounded to 0 or 1 in FP32 are taken at the nearest interior point
                    up = fminf(fmaxf(up, 0x1p-25f), 0x1.fffffep-1f);  // 1 - 2^-24, the largest float below 1
                    const float z = flog(up) - flog(1.0f - up);
                    zr[d] = z;
                    lqp[nt] -= log_sig_prime(z);
                }
            } else {
                const uint64_t idx = a.first + (uint64_t)(valid ? s : 0);
#pragma unroll
                for (int b4 = 0; b4 * 4 < D; ++b4) {
                    if ((b4 & 1) != h) continue;
                    uint32_t c[4] = {(uint32_t)idx, (uint32_t)(idx >> 32), (uint32_t)b4, 0u};
                    philox(c, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
#pragma unroll
                    for (int w = 0; w < 4; ++w) {
                        const int d = 4 * b4 + w;
                        if (d < D) {
                            if (valid && a.u_out) a.u_out[(int64_t)d * a.ld + s] = ((float)(c[w] >> 8) + 0.5f) * 0x1p-24f;
                            if (a.jv_out) {
                                // the sampler's bin: (2m + 1) B >> 25 in integers
                                const uint32_t bin = (uint32_t)(((2ull * (c[w] >> 8) + 1ull) * (uint64_t)a.n_bins) >> 25);
                                const float* e = a.edges + d * (a.n_bins + 1) + bin;
                                jvp[nt] *= (float)a.n_bins * (e[1] - e[0]);
                            }
                            const float z = philox_logit(c[w]);
                            zr[d] = z;
                            lqp[nt] -= log_sig_prime(z);
                        }
                    }
                }
            }
        }
        for (int l = L - 1; l >= 0; --l, ++g) {
            wait_copies();
            __syncthreads();
            if (l > 0 || bt + gridDim.x < nbatch)
                prefetch_layer(sm + ((g + 1) & 1 ? PassLds<D>::buf1 : PassLds<D>::buf0), a.shadow, l > 0 ? l - 1 : L - 1);
            coupling_layer<D, true>(sm + (g & 1 ? PassLds<D>::buf1 : PassLds<D>::buf0), zw, a.aidx + l * 16,
                                    a.bidx + l * 16, a.dA[l], lqp);
            if (a.states)
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) {
                    const int64_t s = base + 32 * nt + j;
                    if (s < a.n)
                        for (int d = h; d < D; d += 2)
                            a.states[((int64_t)l * D + d) * a.n + s] = zw[(32 * nt + j) * ZS + d];
                }
        }
        const int64_t s = base + 32 * h + j;
        const bool valid = s < a.n;
        float lq = lqp[h] + __shfl_xor(lqp[1 - h], 32);
        const float jv = jvp[h] * __shfl_xor(jvp[1 - h], 32);
        if (valid && a.jv_out) a.jv_out[s] = jv;
        const float* zr = zw + (32 * h + j) * ZS;
        for (int d = 0; d < D; ++d) lq += log_sig_prime(zr[d]);
        // a sample whose density is not finite is dropped from the loss and the gradient
        float w = valid && a.w ? (float)((double)a.w[s] * a.inv_wsum[0]) : 0.0f;
        if (!__builtin_isfinite(lq) || !__builtin_isfinite(w)) w = 0.0f;
        if (valid && a.weff) a.weff[s] = w;
        if (valid && a.G)
            for (int d = 0; d < D; ++d) {
                const float sg = fsigmoid(zr[d]);
                a.G[(int64_t)d * a.n + s] = w != 0.0f ? -w * (1.0f - 2.0f * sg) : 0.0f;
            }
        if (valid && a.lq_out) a.lq_out[s] = lq;
        if (valid && w != 0.0f) loss -= w * lq;
    }
    wait_copies();
    // deterministic block loss: wave sums, then waves in order
    for (int o = 32; o > 0; o >>= 1) loss += __shfl_xor(loss, o);
    __shared__ float wl_[PASS_WAVES];
    if (lane == 0) wl_[wv] = loss;
    __syncthreads();
    if (threadIdx.x == 0 && a.loss_part) {
        float t = 0.0f;
        for (int w = 0; w < PASS_WAVES; ++w) t += wl_[w];
        a.loss_part[blockIdx.x] = t;
    }
}

// ---------------------------------------------------------------- training
// Network of one layer for 32 samples (one tile) with weight fragments read from global memory
// (L2-resident); keeps X1, H1, H2 (BF16) in the wave's LDS and returns s_hat, t in O.
struct TrainWave {
    static constexpr int x1 = 0;                     // bf16 [32][XS]
    static constexpr int h1 = x1 + 32 * XS * 2;      // bf16 [32][HS]
    static constexpr int h2 = h1 + 32 * HS * 2;      // bf16 [32][HS]
    static constexpr int dp = h2 + 32 * HS * 2;      // bf16 [32][HS] (dpre2, then dpre1)
    static constexpr int o = dp + 32 * HS * 2;       // f32 [32][OS] (O, then dO as bf16 [32][XS2])
    static constexpr int dx = o + 32 * OS * 4;       // f32 [32][OS] (gradient of X1)
    static constexpr int bytes = dx + 32 * OS * 4;
};
constexpr int XS2 = FNOUT + 8;  // 40: bf16 row stride of dO

__device__ __forceinline__ bf16x8 gfrag(const __bf16* p) { return *(const bf16x8*)p; }

__device__ void tile_mlp_global(const __bf16* wl, const float* ml, char* wb, const float* zrow, const int* aidx,
                                int dA, bool have_row) {
    const int lane = threadIdx.x & 63, h = lane >> 5, col = lane & 31;
    __bf16* x1 = (__bf16*)(wb + TrainWave::x1);
    __bf16* h1 = (__bf16*)(wb + TrainWave::h1);
    __bf16* h2 = (__bf16*)(wb + TrainWave::h2);
    float* ob = (float*)(wb + TrainWave::o);
    // lanes 0..31 own the 32 samples' X1 rows
    if (lane < 32) {
#pragma unroll
        for (int k = 0; k < FKIN; ++k) {
            const float v = (k < dA && have_row) ? fsigmoid(zrow[aidx[k]]) : (k == dA ? 1.0f : 0.0f);
            x1[lane * XS + k] = (__bf16)v;
        }
    }
    wave_sync();
    const bf16x8 bx = *(const bf16x8*)(x1 + col * XS + 8 * h);
#pragma unroll
    for (int ot = 0; ot < 4; ++ot) {
        f32x16 c = {};
        c = mfma(gfrag(wl + SH_W1T + (32 * ot + col) * FKIN + 8 * h), bx, c);
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            bf16x4 v;
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = (__bf16)fmaxf(c[4 * g + q], 0.0f);
            *(bf16x4*)(h1 + col * HS + 32 * ot + 8 * g + 4 * h) = v;
        }
    }
    wave_sync();
    f32x16 acc[4];
#pragma unroll
    for (int ot = 0; ot < 4; ++ot)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[ot][r] = ml[OFF_B2 + 32 * ot + 8 * (r >> 2) + 4 * h + (r & 3)];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const bf16x8 bb = *(const bf16x8*)(h1 + col * HS + 16 * s + 8 * h);
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) acc[ot] = mfma(gfrag(wl + SH_W2T + (32 * ot + col) * FH + 16 * s + 8 * h), bb, acc[ot]);
    }
#pragma unroll
    for (int ot = 0; ot < 4; ++ot)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            bf16x4 v;
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = (__bf16)fmaxf(acc[ot][4 * g + q], 0.0f);
            *(bf16x4*)(h2 + col * HS + 32 * ot + 8 * g + 4 * h) = v;
        }
    wave_sync();
    f32x16 o3;
#pragma unroll
    for (int r = 0; r < 16; ++r) o3[r] = ml[OFF_B3 + 8 * (r >> 2) + 4 * h + (r & 3)];
#pragma unroll
    for (int s = 0; s < 8; ++s)
        o3 = mfma(gfrag(wl + SH_W3T + col * FH + 16 * s + 8 * h), *(const bf16x8*)(h2 + col * HS + 16 * s + 8 * h), o3);
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        f32x4 v;
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = o3[4 * g + q];
        *(f32x4*)(ob + col * OS + 8 * g + 4 * h) = v;
    }
    wave_sync();
}

// One layer of the reverse sweep (layer l, visited in order 0..L-1).
__global__ void __launch_bounds__(256) dmc_flow_bwd_kernel(FlowTrainArgs a, int l) {
    extern __shared__ __attribute__((aligned(16))) char sm[];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, h = lane >> 5, col = lane & 31;
    char* wb = sm + wv * TrainWave::bytes;
    float* zs = (float*)(sm + 4 * TrainWave::bytes) + wv * 32 * ZMAX;
    const int D = a.dim;
    const int dA = a.dA[l], dB = D - dA;
    const __bf16* wl = a.shadow + (size_t)l * SHADOW_LAYER;
    const float* ml = a.master + (size_t)l * LAYER_SIZE;
    const int* aidx = a.aidx + l * 16;
    const int* bidx = a.bidx + l * 16;
    __bf16* x1 = (__bf16*)(wb + TrainWave::x1);
    __bf16* h1 = (__bf16*)(wb + TrainWave::h1);
    __bf16* h2 = (__bf16*)(wb + TrainWave::h2);
    __bf16* dp = (__bf16*)(wb + TrainWave::dp);
    float* ob = (float*)(wb + TrainWave::o);
    __bf16* dob = (__bf16*)(wb + TrainWave::o);
    float* dxb = (float*)(wb + TrainWave::dx);
    const int64_t ntile = (a.n + 31) / 32;
    for (int64_t t = (int64_t)blockIdx.x * 4 + wv; t < ntile; t += (int64_t)gridDim.x * 4) {
        const int64_t s = t * 32 + col;
        const bool valid = s < a.n;
        float* zr = zs + col * ZMAX;
        if (lane < 32)
            for (int d = 0; d < D; ++d) zr[d] = valid ? a.states[((int64_t)l * D + d) * a.n + s] : 0.0f;
        wave_sync();
        tile_mlp_global(wl, ml, wb, zr, aidx, dA, true);
        // coupling backward (lanes 0..31, one sample each): dO = (G_shat, G_t), staged in FP32
        // in the dX buffer (O aliases the BF16 dO buffer)
        if (lane < 32) {
            const float* orow = ob + col * OS;
            float* grow = dxb + col * OS;
            for (int o = 0; o < FNOUT; ++o) grow[o] = 0.0f;
            const float w = valid ? a.weff[s] : 0.0f;
            for (int b = 0; b < dB; ++b) {
                const int zi = bidx[b];
                const float th = ftanh(orow[b]);
                const float sv = FLOW_SMAX * th;
                const float e = fexp(-sv);
                const float gB = valid ? a.G[(int64_t)zi * a.n + s] : 0.0f;
                const float zBo = zr[zi];  // z_B(l), the inverse layer's output
                grow[b] = (-gB * zBo + w) * FLOW_SMAX * (1.0f - th * th);
                grow[16 + b] = -gB * e;
                if (valid) a.G[(int64_t)zi * a.n + s] = gB * e;
            }
        }
        wave_sync();
        if (lane < 32) {
            for (int o = 0; o < FNOUT; ++o) dob[col * XS2 + o] = (__bf16)dxb[col * OS + o];
            for (int o = FNOUT; o < XS2; ++o) dob[col * XS2 + o] = (__bf16)0.0f;
        }
        wave_sync();
        // activations and output gradient to global (feature-major, sample-contiguous) for the
        // weight-gradient products
        if (valid && lane < 32) {
            for (int k = 0; k < FKIN; ++k) a.act_x1[(int64_t)k * a.lda + s] = x1[col * XS + k];
            for (int o = 0; o < FNOUT; ++o) a.act_do[(int64_t)o * a.lda + s] = dob[col * XS2 + o];
        }
        for (int k = h; k < FH; k += 2)
            if (valid) {
                a.act_h1[(int64_t)k * a.lda + s] = h1[col * HS + k];
                a.act_h2[(int64_t)k * a.lda + s] = h2[col * HS + k];
            }
        // dH2^T = W3 dO^T (A = W3 [hidden][out], K = 32 out in 2 steps); mask by H2 > 0 -> dpre2
        f32x16 d2[4];
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) {
            d2[ot] = (f32x16){};
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2)
                d2[ot] = mfma(gfrag(wl + SH_W3 + (32 * ot + col) * FNOUT + 16 * s2 + 8 * h),
                              *(const bf16x8*)(dob + col * XS2 + 16 * s2 + 8 * h), d2[ot]);
        }
        wave_sync();
#pragma unroll
        for (int ot = 0; ot < 4; ++ot)
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                bf16x4 v;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int hid = 32 * ot + 8 * g + 4 * h + q;
                    const float m = (float)h2[col * HS + hid] > 0.0f ? 1.0f : 0.0f;
                    v[q] = (__bf16)(d2[ot][4 * g + q] * m);
                }
                *(bf16x4*)(dp + col * HS + 32 * ot + 8 * g + 4 * h) = v;
            }
        wave_sync();
        for (int k = h; k < FH; k += 2)
            if (valid) a.act_dp2[(int64_t)k * a.lda + s] = dp[col * HS + k];
        // dH1^T = W2 dpre2^T (A = W2 [in hidden][out hidden]); mask by H1 > 0 -> dpre1
        f32x16 d1[4];
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) d1[ot] = (f32x16){};
#pragma unroll
        for (int s2 = 0; s2 < 8; ++s2) {
            const bf16x8 bb = *(const bf16x8*)(dp + col * HS + 16 * s2 + 8 * h);
#pragma unroll
            for (int ot = 0; ot < 4; ++ot)
                d1[ot] = mfma(gfrag(wl + SH_W2 + (32 * ot + col) * FH + 16 * s2 + 8 * h), bb, d1[ot]);
        }
        wave_sync();
#pragma unroll
        for (int ot = 0; ot < 4; ++ot)
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                bf16x4 v;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int hid = 32 * ot + 8 * g + 4 * h + q;
                    const float m = (float)h1[col * HS + hid] > 0.0f ? 1.0f : 0.0f;
                    v[q] = (__bf16)(d1[ot][4 * g + q] * m);
                }
                *(bf16x4*)(dp + col * HS + 32 * ot + 8 * g + 4 * h) = v;
            }
        wave_sync();
        for (int k = h; k < FH; k += 2)
            if (valid) a.act_dp1[(int64_t)k * a.lda + s] = dp[col * HS + k];
        // dX1^T = W1 dpre1^T (A = W1 [32 rows: 16 inputs + zero pad][128])
        f32x16 dx = {};
#pragma unroll
        for (int s2 = 0; s2 < 8; ++s2)
            dx = mfma(gfrag(wl + SH_W1 + col * FH + 16 * s2 + 8 * h), *(const bf16x8*)(dp + col * HS + 16 * s2 + 8 * h), dx);
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            f32x4 v;
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = dx[4 * g + q];
            *(f32x4*)(dxb + col * OS + 8 * g + 4 * h) = v;
        }
        wave_sync();
        if (valid && lane < 32)
            for (int k = 0; k < dA; ++k) {
                const int zi = aidx[k];
                const float sg = fsigmoid(zr[zi]);
                a.G[(int64_t)zi * a.n + s] += dxb[col * OS + k] * sg * (1.0f - sg);
            }
        wave_sync();
    }
}

// Weight gradients of one layer, split over sample chunks: block (c, g) sums the samples of chunk
// c, [c * chunk, (c + 1) * chunk), in a fixed order into partial[c][LAYER_SIZE]; group g picks the
// output: g = 0..3 the W2t row block g (wave w: column block w), g = 4 W1t (wave w: row block w),
// g = 5 W3t (wave w: column block w), g = 6 the biases.  The four waves of a W2t block read the
// same dpre2 rows at the same time, so those loads are served once from the CU's cache.
//   W1t[h][k] = sum_s dpre1[h][s] X1[k][s]
//   W2t[o][i] = sum_s dpre2[o][s] H1[i][s]
//   W3t[o][i] = sum_s dO[o][s]    H2[i][s]
//   b2[o] = sum_s dpre2[o][s],  b3[o] = sum_s dO[o][s]   (FP32, in sample order)
// Activation rows have stride lda (a multiple of 16 samples): every 16-sample slice of a row is one
// aligned pair of 16-byte loads; slices past the chunk end are masked to zero.
__device__ __forceinline__ bf16x8 masked_slice(const __bf16* row, int64_t k, int64_t s1, bool ok) {
    bf16x8 v = {};
    if (ok) {
        v = *(const bf16x8*)(row + k);
        if (k + 8 > s1)
#pragma unroll
            for (int t = 0; t < 8; ++t)
                if (k + t >= s1) v[t] = (__bf16)0.0f;
    }
    return v;
}

__global__ void __launch_bounds__(256) dmc_flow_wgrad_kernel(FlowTrainArgs a, int chunk, float* partial) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, h = lane >> 5, col = lane & 31;
    const int g = blockIdx.y;
    const int64_t s0 = (int64_t)blockIdx.x * chunk;
    const int64_t s1 = min(s0 + (int64_t)chunk, a.n);
    float* out = partial + (size_t)blockIdx.x * LAYER_SIZE;
    if (g == 6) {
        // bias gradients: sums of the rounded output gradients in sample order
        const int r = threadIdx.x;
        if (r < FH + FNOUT) {
            const __bf16* src = r < FH ? a.act_dp2 + (int64_t)r * a.lda : a.act_do + (int64_t)(r - FH) * a.lda;
            float acc = 0.0f;
            for (int64_t k = s0; k < s1; k += 8) {
                const bf16x8 v = masked_slice(src, k, s1, true);
#pragma unroll
                for (int t = 0; t < 8; ++t) acc += (float)v[t];
            }
            if (r < FH)
                out[OFF_B2 + r] = acc;
            else
                out[OFF_B3 + r - FH] = acc;
        }
        return;
    }
    const __bf16* Ab;
    const __bf16* Bb;
    int rows_base, cols_base, ncols, ld_dst;
    float* dst;
    if (g < 4) {
        Ab = a.act_dp2 + (int64_t)(32 * g) * a.lda;
        Bb = a.act_h1 + (int64_t)(32 * wv) * a.lda;
        rows_base = 32 * g;
        cols_base = 32 * wv;
        ncols = 32;
        dst = out + OFF_W2T;
        ld_dst = FH;
    } else if (g == 4) {
        Ab = a.act_dp1 + (int64_t)(32 * wv) * a.lda;
        Bb = a.act_x1;
        rows_base = 32 * wv;
        cols_base = 0;
        ncols = FKIN;
        dst = out + OFF_W1T;
        ld_dst = FKIN;
    } else {
        Ab = a.act_do;
        Bb = a.act_h2 + (int64_t)(32 * wv) * a.lda;
        rows_base = 0;
        cols_base = 32 * wv;
        ncols = 32;
        dst = out + OFF_W3T;
        ld_dst = FH;
    }
    const bool bok = col < ncols;
    const __bf16* Ar = Ab + (int64_t)col * a.lda;
    const __bf16* Br = Bb + (int64_t)(bok ? col : 0) * a.lda;
    f32x16 c0 = {}, c1 = {};
    for (int64_t k0 = s0; k0 < s1; k0 += 64) {
        bf16x8 av[4], bv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t k = k0 + 16 * u + 8 * h;
            const bool in = k0 + 16 * u < s1;
            av[u] = masked_slice(Ar, k, s1, in);
            bv[u] = masked_slice(Br, k, s1, in && bok);
        }
        c0 = mfma(av[0], bv[0], c0);
        c1 = mfma(av[1], bv[1], c1);
        c0 = mfma(av[2], bv[2], c0);
        c1 = mfma(av[3], bv[3], c1);
    }
    if (bok)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = rows_base + 8 * (r >> 2) + 4 * h + (r & 3);
            dst[row * ld_dst + cols_base + col] = c0[r] + c1[r];
        }
}

// Fold the per-block partial gradients (fixed order, FP64), scale by 1/sum(w), Adam on the FP32
// masters (Kingma and Ba 2015, bias-corrected), and refresh the BF16 shadows.  Also folds the
// partial losses and sum(w) (thread 0 of block 0).
__global__ void __launch_bounds__(256) dmc_flow_adam_kernel(FlowAdamArgs a) {
    const int64_t P = (int64_t)a.n_layers * LAYER_SIZE;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
        const int l = (int)(p / LAYER_SIZE);
        const int q = (int)(p % LAYER_SIZE);
        double g = 0.0;
        const float* src = a.partial + (size_t)l * a.nblk_max * LAYER_SIZE + q;
        for (int b = 0; b < a.nblk; ++b) g += (double)src[(size_t)b * LAYER_SIZE];
        if (a.grad_out) a.grad_out[p] = (float)g;
        if (!a.apply || !isfinite(g)) continue;
        float th = a.master[p];
        float m = a.m[p] = (float)(a.b1 * a.m[p] + (1.0 - a.b1) * g);
        float v = a.v[p] = (float)(a.b2 * a.v[p] + (1.0 - a.b2) * g * g);
        const double mh = m / (1.0 - a.b1t), vh = v / (1.0 - a.b2t);
        th = (float)(th - a.lr * mh / (sqrt(vh) + a.eps));
        a.master[p] = th;
        write_shadow(a.shadow, l, q, th);
    }
}

// samples drawn from the grid alone: J <- J / (alpha q_flow + 1 - alpha)
// balance-heuristic weight of points drawn from one share of the mixture
__global__ void dmc_flow_mix_kernel(float* jac, const float* lq, const float* jv, int64_t n, float a_f, float a_g,
                                    float a_u, int scale_jv) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float v = jv[i];
        const float den = __builtin_fmaf(a_f, fexp(lq[i]), __builtin_fmaf(a_u, v, a_g));
        jac[i] = (scale_jv ? jac[i] * v : jac[i]) / den;
    }
}

// The uniform share: Philox y (24-bit uniform), physical map, u' = G^-1(y) by a binary search of
// the grid edges (the bin b with e_b <= y < e_{b+1}, clamped to the grid), J_V = prod_d B (e_{b+1} - e_b).
__global__ void __launch_bounds__(256) dmc_flow_uniform_kernel(FlowUniformArgs a) {
    const int D = a.dim, B = a.n_bins, N = (D + 1) / 4;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < a.n; s += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t idx = a.first + (uint64_t)s;
        float jv = 1.0f, jp = a.jt;
        float y[ZMAX];
        for (int b4 = 0; b4 * 4 < D; ++b4) {
            uint32_t c[4] = {(uint32_t)idx, (uint32_t)(idx >> 32), (uint32_t)b4, 0u};
            philox(c, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
            for (int w = 0; w < 4 && 4 * b4 + w < D; ++w) y[4 * b4 + w] = ((float)(c[w] >> 8) + 0.5f) * 0x1p-24f;
        }
        for (int d = 0; d < D; ++d) {
            const float* e = a.edges + d * (B + 1);
            int lo = 0, hi = B;  // invariant: e[lo] <= y, answer in [lo, hi)
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (e[mid] <= y[d])
                    lo = mid;
                else
                    hi = mid;
            }
            const float w = e[lo + 1] - e[lo];
            const float fr = w > 0.0f ? fminf((y[d] - e[lo]) / w, 1.0f) : 0.0f;
            a.u_out[(int64_t)d * a.ldu + s] = ((float)lo + fr) / (float)B;
            jv *= (float)B * w;
        }
        for (int q = 0; q < N; ++q) {
            const float r = a.qmax * y[3 * q];
            const float ct = __builtin_fmaf(2.0f, y[3 * q + 1], -1.0f);
            const float st = __builtin_sqrtf(__builtin_fmaxf(0.0f, __builtin_fmaf(-ct, ct, 1.0f)));
            float sp, cp;
            sincospif(2.0f * y[3 * q + 2], &sp, &cp);
            a.x[(int64_t)(3 * q) * a.ld + s] = r * st * cp;
            a.x[(int64_t)(3 * q + 1) * a.ld + s] = r * st * sp;
            a.x[(int64_t)(3 * q + 2) * a.ld + s] = r * ct;
            jp *= a.jl * r * r;
        }
        for (int j = 1; j < N; ++j) a.x[(int64_t)(3 * N + j - 1) * a.ld + s] = a.beta * y[3 * N + j - 1];
        a.jac[s] = jp;
        a.jv_out[s] = jv;
    }
}

__global__ void __launch_bounds__(256) dmc_flow_shadow_kernel(const float* master, __bf16* shadow, int n_layers) {
    const int64_t P = (int64_t)n_layers * LAYER_SIZE;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x)
        write_shadow(shadow, (int)(p / LAYER_SIZE), (int)(p % LAYER_SIZE), master[p]);
}

// sum of w in a fixed order (one block): out[0] = sum, out[2] = 1 / sum (0 if the sum is not
// positive and finite); the normalised loss is folded by dmc_flow_loss_kernel after the pass
__global__ void __launch_bounds__(1024) dmc_flow_sums_kernel(const float* w, int64_t n, double* out) {
    __shared__ double red[1024];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) acc += (double)w[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = red[0];
        out[2] = (red[0] > 0.0 && red[0] < 1e300) ? 1.0 / red[0] : 0.0;
    }
}

__global__ void dmc_flow_loss_kernel(const float* loss_part, int nblk, double* out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double L = 0.0;
        for (int b = 0; b < nblk; ++b) L += (double)loss_part[b];
        out[1] = L;
    }
}

// ---------------------------------------------------------------- launchers
// Sampler and inverse: one 512-thread block per CU (grid-stride over batches of 512 samples)
static int pass_blocks(int64_t n, int n_cu) {
    const int64_t want = (n + PASS_THREADS - 1) / PASS_THREADS;
    return (int)(want < (int64_t)n_cu ? want : (int64_t)n_cu);
}

template <int D>
static hipError_t launch_sample_d(const FlowSampleArgs& a, int n_cu, hipStream_t st) {
    constexpr int smem = PassLds<D>::bytes;
    hipError_t e = hipFuncSetAttribute((const void*)dmc_flow_sample_kernel<D>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, smem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(dmc_flow_sample_kernel<D>, dim3(pass_blocks(a.n, n_cu)), dim3(PASS_THREADS), smem, st, a);
    return hipGetLastError();
}

int flow_sample_lds_bytes(int dim) {
    switch (dim) {
        case 3: return PassLds<3>::bytes;
        case 7: return PassLds<7>::bytes;
        case 11: return PassLds<11>::bytes;
        case 15: return PassLds<15>::bytes;
        case 19: return PassLds<19>::bytes;
        case 23: return PassLds<23>::bytes;
    }
    return -1;
}

hipError_t launch_flow_sample(const FlowSampleArgs& a, int dim, int n_cu, hipStream_t st) {
    switch (dim) {
        case 3: return launch_sample_d<3>(a, n_cu, st);
        case 7: return launch_sample_d<7>(a, n_cu, st);
        case 11: return launch_sample_d<11>(a, n_cu, st);
        case 15: return launch_sample_d<15>(a, n_cu, st);
        case 19: return launch_sample_d<19>(a, n_cu, st);
        case 23: return launch_sample_d<23>(a, n_cu, st);
    }
    return hipErrorInvalidValue;
}

constexpr int TRAIN_LDS = 4 * TrainWave::bytes + 4 * 32 * ZMAX * 4;

int flow_train_blocks(int64_t n, int n_cu) {
    const int64_t tiles = (n + 31) / 32;
    const int64_t want = (tiles + 3) / 4;
    return (int)(want < (int64_t)n_cu * 2 ? want : (int64_t)n_cu * 2);
}

int flow_inverse_blocks(int64_t n, int n_cu) { return pass_blocks(n, n_cu); }

template <int D>
static hipError_t launch_inverse_d(const FlowTrainArgs& a, int nblk, hipStream_t st) {
    constexpr int smem = PassLds<D>::bytes;
    hipError_t e = hipFuncSetAttribute((const void*)dmc_flow_inverse_kernel<D>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, smem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(dmc_flow_inverse_kernel<D>, dim3(nblk), dim3(PASS_THREADS), smem, st, a);
    return hipGetLastError();
}

hipError_t launch_flow_inverse(const FlowTrainArgs& a, int nblk, hipStream_t st) {
    switch (a.dim) {
        case 3: return launch_inverse_d<3>(a, nblk, st);
        case 7: return launch_inverse_d<7>(a, nblk, st);
        case 11: return launch_inverse_d<11>(a, nblk, st);
        case 15: return launch_inverse_d<15>(a, nblk, st);
        case 19: return launch_inverse_d<19>(a, nblk, st);
        case 23: return launch_inverse_d<23>(a, nblk, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_flow_backward(const FlowTrainArgs& a, int nblk, int layer, int wg_chunk, int wg_blocks,
                                float* partial_layer, hipStream_t st) {
    hipError_t e = hipFuncSetAttribute((const void*)dmc_flow_bwd_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       TRAIN_LDS);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(dmc_flow_bwd_kernel, dim3(nblk), dim3(256), TRAIN_LDS, st, a, layer);
    hipLaunchKernelGGL(dmc_flow_wgrad_kernel, dim3(wg_blocks, 7), dim3(256), 0, st, a, wg_chunk, partial_layer);
    return hipGetLastError();
}

hipError_t launch_flow_sums(const float* w, int64_t n, double* out, hipStream_t st) {
    hipLaunchKernelGGL(dmc_flow_sums_kernel, dim3(1), dim3(1024), 0, st, w, n, out);
    return hipGetLastError();
}

hipError_t launch_flow_loss(const float* loss_part, int nblk, double* out, hipStream_t st) {
    hipLaunchKernelGGL(dmc_flow_loss_kernel, dim3(1), dim3(64), 0, st, loss_part, nblk, out);
    return hipGetLastError();
}

hipError_t launch_flow_adam(const FlowAdamArgs& a, int n_cu, hipStream_t st) {
    hipLaunchKernelGGL(dmc_flow_adam_kernel, dim3(n_cu * 4), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_flow_mix(float* jac, const float* lq, const float* jv, int64_t n, float a_f, float a_g, float a_u,
                           bool scale_jv, hipStream_t st) {
    const int64_t want = (n + 255) / 256;
    hipLaunchKernelGGL(dmc_flow_mix_kernel, dim3((unsigned)(want < 4096 ? want : 4096)), dim3(256), 0, st, jac, lq, jv,
                       n, a_f, a_g, a_u, scale_jv ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_flow_uniform(const FlowUniformArgs& a, int n_cu, hipStream_t st) {
    const int64_t want = (a.n + 255) / 256;
    const int64_t cap = (int64_t)n_cu * 8;
    hipLaunchKernelGGL(dmc_flow_uniform_kernel, dim3((unsigned)(want < cap ? want : cap)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_flow_shadow(const float* master, __bf16* shadow, int n_layers, int n_cu, hipStream_t st) {
    hipLaunchKernelGGL(dmc_flow_shadow_kernel, dim3(n_cu * 4), dim3(256), 0, st, master, shadow, n_layers);
    return hipGetLastError();
}

}  // namespace dmc
