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

// log sigma'(z) = -|z| - 2 log(1 + e^{-|z|})
__device__ __forceinline__ float log_sig_prime(float z) {
    const float a = fabsf(z);
    return -a - 2.0f * log1pf(expf(-a));
}

// logit of the 24-bit uniform u = (m + 1/2) 2^-24, m = w >> 8: log(m + 1/2) - log(2^24 - 1 - m + 1/2).
// Both operands are exact in FP32 wherever their logarithm is sensitive to rounding (below 2^23),
// so the result is finite for every word (u itself rounds to 1 in FP32 at m = 2^24 - 1).
__device__ __forceinline__ float philox_logit(uint32_t w) {
    const uint32_t m = w >> 8;
    return logf((float)m + 0.5f) - logf((float)(0xFFFFFFu - m) + 0.5f);
}

// ---------------------------------------------------------------- LDS geometry
// Row strides padded by 8 BF16 (16 B) so that 16 lanes reading 16 B each hit distinct banks.
constexpr int W1S = FKIN + 8;   // 24
constexpr int W2S = FH + 8;     // 136
constexpr int XS = FKIN + 8;    // 24
constexpr int HS = FH + 8;      // 136
constexpr int OS = FNOUT + 4;   // 36 floats

struct FwdLds {
    static constexpr int w1t = 0;                           // bf16 [128][W1S]
    static constexpr int w2t = w1t + FH * W1S * 2;          // bf16 [128][W2S]
    static constexpr int w3t = w2t + FH * W2S * 2;          // bf16 [32][W2S]
    static constexpr int b2 = w3t + FNOUT * W2S * 2;        // f32 [128]
    static constexpr int b3 = b2 + FH * 4;                  // f32 [32]
    static constexpr int idx = b3 + FNOUT * 4;              // int [32]: a list (16), b list (16)
    static constexpr int waves = idx + 32 * 4;              // per-wave regions
};

template <int D>
struct WaveLds {
    static constexpr int ZS = D + 2;                        // odd row stride of the state rows
    static constexpr int x1 = 0;                            // bf16 [64][XS]
    static constexpr int h = x1 + 64 * XS * 2;              // bf16 [64][HS]; f32 [64][OS] aliases it
    static constexpr int z = h + 64 * HS * 2;               // f32 [64][ZS]
    static constexpr int bytes = z + 64 * ZS * 4;
};

template <int D>
constexpr int flow_fwd_lds_bytes() {
    return FwdLds::waves + 4 * WaveLds<D>::bytes;
}

// stage the forward weights of one layer (global bf16 shadow, unpadded rows) into padded LDS rows
__device__ void stage_fwd(char* sm, const __bf16* shadow, const float* master, const int* aidx, const int* bidx,
                          int layer) {
    const __bf16* wl = shadow + (size_t)layer * SHADOW_LAYER;
    const float* ml = master + (size_t)layer * LAYER_SIZE;
    __bf16* w1t = (__bf16*)(sm + FwdLds::w1t);
    __bf16* w2t = (__bf16*)(sm + FwdLds::w2t);
    __bf16* w3t = (__bf16*)(sm + FwdLds::w3t);
    // 16-byte chunks: W1t 128 rows x 2, W2t 128 x 16, W3t 32 x 16
    for (int c = threadIdx.x; c < FH * 2 + FH * 16 + FNOUT * 16; c += blockDim.x) {
        if (c < FH * 2) {
            const int r = c >> 1, k = (c & 1) * 8;
            *(uint4*)(w1t + r * W1S + k) = *(const uint4*)(wl + SH_W1T + r * FKIN + k);
        } else if (c < FH * 2 + FH * 16) {
            const int cc = c - FH * 2, r = cc >> 4, k = (cc & 15) * 8;
            *(uint4*)(w2t + r * W2S + k) = *(const uint4*)(wl + SH_W2T + r * FH + k);
        } else {
            const int cc = c - FH * 2 - FH * 16, r = cc >> 4, k = (cc & 15) * 8;
            *(uint4*)(w3t + r * W2S + k) = *(const uint4*)(wl + SH_W3T + r * FH + k);
        }
    }
    float* b2 = (float*)(sm + FwdLds::b2);
    float* b3 = (float*)(sm + FwdLds::b3);
    int* ix = (int*)(sm + FwdLds::idx);
    for (int i = threadIdx.x; i < FH + FNOUT + 32; i += blockDim.x) {
        if (i < FH)
            b2[i] = ml[OFF_B2 + i];
        else if (i < FH + FNOUT)
            b3[i - FH] = ml[OFF_B3 + i - FH];
        else {
            const int j = i - FH - FNOUT;
            ix[j] = j < 16 ? aidx[layer * 16 + j] : bidx[layer * 16 + j - 16];
        }
    }
}

// The network of one coupling layer for the wave's 64 samples (two 32-sample tiles).  On return
// the wave's O buffer (f32 [64][OS], aliasing H) holds s_hat (columns 0..15) and t (16..31).
template <int D>
__device__ void wave_mlp_lds(char* sm, char* wb, int dA) {
    const int lane = threadIdx.x & 63, h = lane >> 5, col = lane & 31;
    const __bf16* w1t = (const __bf16*)(sm + FwdLds::w1t);
    const __bf16* w2t = (const __bf16*)(sm + FwdLds::w2t);
    const __bf16* w3t = (const __bf16*)(sm + FwdLds::w3t);
    const float* b2 = (const float*)(sm + FwdLds::b2);
    const float* b3 = (const float*)(sm + FwdLds::b3);
    const int* ix = (const int*)(sm + FwdLds::idx);
    __bf16* x1 = (__bf16*)(wb + WaveLds<D>::x1);
    __bf16* hb = (__bf16*)(wb + WaveLds<D>::h);
    float* ob = (float*)(wb + WaveLds<D>::h);
    const float* zr = (const float*)(wb + WaveLds<D>::z) + lane * WaveLds<D>::ZS;

    // X1 row of this lane's sample: sigmoid(z_A), then the constant 1 that carries the first-layer bias
#pragma unroll
    for (int k = 0; k < FKIN; ++k) {
        const float v = k < dA ? 1.0f / (1.0f + expf(-zr[ix[k]])) : (k == dA ? 1.0f : 0.0f);
        x1[lane * XS + k] = (__bf16)v;
    }
    wave_sync();
    // layer 1: 4 output tiles x 2 sample tiles, K = 16
    bf16x8 bx[2];
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) bx[nt] = *(const bf16x8*)(x1 + (32 * nt + col) * XS + 8 * h);
#pragma unroll
    for (int ot = 0; ot < 4; ++ot) {
        const bf16x8 aw = *(const bf16x8*)(w1t + (32 * ot + col) * W1S + 8 * h);
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            f32x16 c = {};
            c = mfma(aw, bx[nt], c);
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                bf16x4 v;
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] = (__bf16)fmaxf(c[4 * g + q], 0.0f);
                *(bf16x4*)(hb + (32 * nt + col) * HS + 32 * ot + 8 * g + 4 * h) = v;
            }
        }
    }
    wave_sync();
    // layer 2: K = 128 in 8 steps of 16; accumulators start at the bias
    f32x16 acc[2][4];
#pragma unroll
    for (int ot = 0; ot < 4; ++ot)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const float bv = b2[32 * ot + 8 * (r >> 2) + 4 * h + (r & 3)];
            acc[0][ot][r] = bv;
            acc[1][ot][r] = bv;
        }
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        bf16x8 bb[2];
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) bb[nt] = *(const bf16x8*)(hb + (32 * nt + col) * HS + 16 * s + 8 * h);
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) {
            const bf16x8 aw = *(const bf16x8*)(w2t + (32 * ot + col) * W2S + 16 * s + 8 * h);
            acc[0][ot] = mfma(aw, bb[0], acc[0][ot]);
            acc[1][ot] = mfma(aw, bb[1], acc[1][ot]);
        }
    }
    wave_sync();
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int ot = 0; ot < 4; ++ot)
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                bf16x4 v;
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] = (__bf16)fmaxf(acc[nt][ot][4 * g + q], 0.0f);
                *(bf16x4*)(hb + (32 * nt + col) * HS + 32 * ot + 8 * g + 4 * h) = v;
            }
    wave_sync();
    // layer 3: 32 outputs, K = 128
    f32x16 o3[2];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const float bv = b3[8 * (r >> 2) + 4 * h + (r & 3)];
        o3[0][r] = bv;
        o3[1][r] = bv;
    }
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const bf16x8 aw = *(const bf16x8*)(w3t + col * W2S + 16 * s + 8 * h);
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const bf16x8 bb = *(const bf16x8*)(hb + (32 * nt + col) * HS + 16 * s + 8 * h);
            o3[nt] = mfma(aw, bb, o3[nt]);
        }
    }
    wave_sync();
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            f32x4 v;
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = o3[nt][4 * g + q];
            *(f32x4*)(ob + (32 * nt + col) * OS + 8 * g + 4 * h) = v;
        }
    wave_sync();
}

template <int D>
__global__ void __launch_bounds__(256) dmc_flow_sample_kernel(FlowSampleArgs a) {
    extern __shared__ __attribute__((aligned(16))) char sm[];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    char* wb = sm + FwdLds::waves + wv * WaveLds<D>::bytes;
    float* zr = (float*)(wb + WaveLds<D>::z) + lane * WaveLds<D>::ZS;
    const float* orow = (const float*)(wb + WaveLds<D>::h) + lane * OS;
    const int* ix = (const int*)(sm + FwdLds::idx);
    constexpr int N = (D + 1) / 4;  // loop momenta
    const int64_t nbatch = (a.n + 255) / 256;
    for (int64_t bt = blockIdx.x; bt < nbatch; bt += gridDim.x) {
        const int64_t s = bt * 256 + threadIdx.x;
        const bool valid = s < a.n;
        const uint64_t idx = a.first + (uint64_t)(valid ? s : 0);
        float lq = 0.0f;
#pragma unroll
        for (int b4 = 0; b4 * 4 < D; ++b4) {
            uint32_t c[4] = {(uint32_t)idx, (uint32_t)(idx >> 32), (uint32_t)b4, 0u};
            philox(c, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const int d = 4 * b4 + w;
                if (d < D) {
                    const float z = philox_logit(c[w]);
                    zr[d] = z;
                    lq += log_sig_prime(z);
                }
            }
        }
        for (int l = 0; l < a.n_layers; ++l) {
            __syncthreads();
            stage_fwd(sm, a.shadow, a.master, a.aidx, a.bidx, l);
            __syncthreads();
            const int dA = a.dA[l], dB = D - dA;
            wave_mlp_lds<D>(sm, wb, dA);
            for (int b = 0; b < dB; ++b) {
                const float sv = FLOW_SMAX * tanhf(orow[b]);
                const int zi = ix[16 + b];
                zr[zi] = zr[zi] * expf(sv) + orow[16 + b];
                lq -= sv;
            }
        }
        if (valid) {
            // u' = sigmoid(z_K); VEGAS map with the bin taken in FP32; physical map
            float J = 1.0f;
            float y[D];
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const float z = zr[d];
                lq -= log_sig_prime(z);
                const float up = 1.0f / (1.0f + expf(-z));
                if (a.u_out) a.u_out[(int64_t)d * a.ld + s] = up;
                const float ub = up * (float)a.n_bins;
                // clamp before the conversion: a non-finite output must not index outside the grid
                const int bin = (int)fminf(fmaxf(ub, 0.0f), (float)(a.n_bins - 1));
                const float fr = ub - (float)bin;
                const float lo = a.edges[d * (a.n_bins + 1) + bin];
                const float hi = a.edges[d * (a.n_bins + 1) + bin + 1];
                y[d] = __builtin_fmaf(fr, hi - lo, lo);
                J *= (float)a.n_bins * (hi - lo);
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
            for (int j = 1; j < N; ++j) a.x[(int64_t)(3 * N + j - 1) * a.ld + s] = a.beta * y[3 * N + j - 1];
            // weight against the mixture density alpha q_flow + (1 - alpha): bounded by the grid's
            // own Jacobian / (1 - alpha) in the flow's tails
            a.jac[s] = J * a.jt / __builtin_fmaf(a.alpha, expf(lq), 1.0f - a.alpha);
            if (a.lq_out) a.lq_out[s] = lq;
        }
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
            const float v = (k < dA && have_row) ? 1.0f / (1.0f + expf(-zrow[aidx[k]])) : (k == dA ? 1.0f : 0.0f);
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

// Inverse pass u' -> z_0 for one sample per lane of the wave's first 32 lanes (tile of 32).
// states[l][d][n]: z^(l) (the output of inverse layer l); lq[n]; G[d][n] = d(-w lq)/dz_0 (unnormalised);
// partial loss per block.
__global__ void __launch_bounds__(256) dmc_flow_inverse_kernel(FlowTrainArgs a) {
    extern __shared__ __attribute__((aligned(16))) char sm[];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    char* wb = sm + wv * TrainWave::bytes;
    float* zs = (float*)(sm + 4 * TrainWave::bytes) + wv * 32 * ZMAX;
    const int D = a.dim;
    float loss = 0.0f;
    const int64_t ntile = (a.n + 31) / 32;
    for (int64_t t = (int64_t)blockIdx.x * 4 + wv; t < ntile; t += (int64_t)gridDim.x * 4) {
        const int64_t s = t * 32 + (lane & 31);
        const bool valid = lane < 32 && s < a.n;
        float* zr = zs + (lane & 31) * ZMAX;
        float lq = 0.0f;
        if (lane < 32) {
            for (int d = 0; d < D; ++d) {
                float up, z;
                if (a.u_in) {
                    up = valid ? a.u_in[(int64_t)d * a.ld + s] : 0.5f;
                    // outputs that rounded to 0 or 1 in FP32 are taken at the nearest interior point
                    up = fminf(fmaxf(up, 0x1p-25f), 0x1.fffffep-1f);  // 1 - 2^-24, the largest float below 1
                    z = logf(up) - log1pf(-up);
                } else {
                    const uint64_t idx = a.first + (uint64_t)(valid ? s : 0);
                    uint32_t c[4] = {(uint32_t)idx, (uint32_t)(idx >> 32), (uint32_t)(d >> 2), 0u};
                    philox(c, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
                    up = ((float)(c[d & 3] >> 8) + 0.5f) * 0x1p-24f;
                    z = philox_logit(c[d & 3]);
                }
                if (valid && a.u_out) a.u_out[(int64_t)d * a.ld + s] = up;
                zr[d] = z;
                lq -= log_sig_prime(z);
            }
        }
        wave_sync();
        for (int l = a.n_layers - 1; l >= 0; --l) {
            const int dA = a.dA[l];
            tile_mlp_global(a.shadow + (size_t)l * SHADOW_LAYER, a.master + (size_t)l * LAYER_SIZE, wb, zr,
                            a.aidx + l * 16, dA, lane < 32);
            const float* orow = (const float*)(wb + TrainWave::o) + (lane & 31) * OS;
            if (lane < 32) {
                for (int b = 0; b < D - dA; ++b) {
                    const float sv = FLOW_SMAX * tanhf(orow[b]);
                    const int zi = a.bidx[l * 16 + b];
                    zr[zi] = (zr[zi] - orow[16 + b]) * expf(-sv);
                    lq -= sv;
                }
                if (valid && a.states)
                    for (int d = 0; d < D; ++d) a.states[((int64_t)l * D + d) * a.n + s] = zr[d];
            }
            wave_sync();
        }
        if (lane < 32) {
            for (int d = 0; d < D; ++d) lq += log_sig_prime(zr[d]);
            // a sample whose density is not finite is dropped from the loss and the gradient
            float w = valid && a.w ? (float)((double)a.w[s] * a.inv_wsum[0]) : 0.0f;
            if (!__builtin_isfinite(lq) || !__builtin_isfinite(w)) w = 0.0f;
            if (valid && a.weff) a.weff[s] = w;
            if (valid && a.G)
                for (int d = 0; d < D; ++d) {
                    const float sg = 1.0f / (1.0f + expf(-zr[d]));
                    a.G[(int64_t)d * a.n + s] = w != 0.0f ? -w * (1.0f - 2.0f * sg) : 0.0f;
                }
            if (valid && a.lq_out) a.lq_out[s] = lq;
            if (valid && w != 0.0f) loss -= w * lq;
        }
        wave_sync();
    }
    // deterministic block loss: wave sums, then waves in order
    for (int o = 32; o > 0; o >>= 1) loss += __shfl_xor(loss, o);
    __shared__ float wl_[4];
    if (lane == 0) wl_[wv] = loss;
    __syncthreads();
    if (threadIdx.x == 0 && a.loss_part) a.loss_part[blockIdx.x] = ((wl_[0] + wl_[1]) + wl_[2]) + wl_[3];
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
                const float th = tanhf(orow[b]);
                const float sv = FLOW_SMAX * th;
                const float e = expf(-sv);
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
            for (int k = 0; k < FKIN; ++k) a.act_x1[(int64_t)k * a.n + s] = x1[col * XS + k];
            for (int o = 0; o < FNOUT; ++o) a.act_do[(int64_t)o * a.n + s] = dob[col * XS2 + o];
        }
        for (int k = h; k < FH; k += 2)
            if (valid) {
                a.act_h1[(int64_t)k * a.n + s] = h1[col * HS + k];
                a.act_h2[(int64_t)k * a.n + s] = h2[col * HS + k];
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
            if (valid) a.act_dp2[(int64_t)k * a.n + s] = dp[col * HS + k];
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
            if (valid) a.act_dp1[(int64_t)k * a.n + s] = dp[col * HS + k];
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
                const float sg = 1.0f / (1.0f + expf(-zr[zi]));
                a.G[(int64_t)zi * a.n + s] += dxb[col * OS + k] * sg * (1.0f - sg);
            }
        wave_sync();
    }
}

// Weight gradients of one layer, split over sample chunks: block b sums samples
// [b * chunk, (b + 1) * chunk) in a fixed order and writes partial[b][LAYER_SIZE].
//   W1t[h][k] = sum_s dpre1[h][s] X1[k][s]   (16 x 128 -> 4 tiles of rows, 1 tile of columns)
//   W2t[o][i] = sum_s dpre2[o][s] H1[i][s]   (16 tiles)
//   W3t[o][i] = sum_s dO[o][s]    H2[i][s]   (4 tiles)
//   b2[o] = sum_s dpre2[o][s],  b3[o] = sum_s dO[o][s]
__global__ void __launch_bounds__(256) dmc_flow_wgrad_kernel(FlowTrainArgs a, int chunk, float* partial) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, h = lane >> 5, col = lane & 31;
    const int64_t s0 = (int64_t)blockIdx.x * chunk;
    const int64_t s1 = min(s0 + (int64_t)chunk, a.n);
    float* out = partial + (size_t)blockIdx.x * LAYER_SIZE;
    // 24 output tiles: 0..15 W2t (row tile rt, column tile ct), 16..19 W1t (rows), 20..23 W3t (cols)
    for (int tile = wv; tile < 24; tile += 4) {
        const __bf16* Ab;
        const __bf16* Bb;
        int rows_base, cols_base, ncols;
        float* dst;
        int ld_dst;
        if (tile < 16) {
            Ab = a.act_dp2 + (int64_t)(32 * (tile >> 2)) * a.n;
            Bb = a.act_h1 + (int64_t)(32 * (tile & 3)) * a.n;
            rows_base = 32 * (tile >> 2);
            cols_base = 32 * (tile & 3);
            ncols = 32;
            dst = out + OFF_W2T;
            ld_dst = FH;
        } else if (tile < 20) {
            Ab = a.act_dp1 + (int64_t)(32 * (tile - 16)) * a.n;
            Bb = a.act_x1;
            rows_base = 32 * (tile - 16);
            cols_base = 0;
            ncols = FKIN;
            dst = out + OFF_W1T;
            ld_dst = FKIN;
        } else {
            Ab = a.act_do;
            Bb = a.act_h2 + (int64_t)(32 * (tile - 20)) * a.n;
            rows_base = 0;
            cols_base = 32 * (tile - 20);
            ncols = 32;
            dst = out + OFF_W3T;
            ld_dst = FH;
        }
        f32x16 c = {};
        const bool bok = col < ncols;
        for (int64_t k0 = s0; k0 < s1; k0 += 16) {
            bf16x8 av, bv;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int64_t k = k0 + 8 * h + t;
                const bool in = k < s1;
                av[t] = in ? Ab[(int64_t)col * a.n + k] : (__bf16)0.0f;
                bv[t] = (in && bok) ? Bb[(int64_t)col * a.n + k] : (__bf16)0.0f;
            }
            c = mfma(av, bv, c);
        }
        if (bok)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = rows_base + 8 * (r >> 2) + 4 * h + (r & 3);
                dst[row * ld_dst + cols_base + col] = c[r];
            }
    }
    // bias gradients: sums of the rounded output gradients in sample order
    for (int r = threadIdx.x; r < FH + FNOUT; r += blockDim.x) {
        const __bf16* src = r < FH ? a.act_dp2 + (int64_t)r * a.n : a.act_do + (int64_t)(r - FH) * a.n;
        float acc = 0.0f;
        for (int64_t k = s0; k < s1; ++k) acc += (float)src[k];
        if (r < FH)
            out[OFF_B2 + r] = acc;
        else
            out[OFF_B3 + r - FH] = acc;
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
__global__ void dmc_flow_mix_kernel(float* jac, const float* lq, int64_t n, float alpha) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        jac[i] = jac[i] / __builtin_fmaf(alpha, expf(lq[i]), 1.0f - alpha);
}

__global__ void __launch_bounds__(256) dmc_flow_shadow_kernel(const float* master, __bf16* shadow, int n_layers) {
    const int64_t P = (int64_t)n_layers * LAYER_SIZE;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x)
        write_shadow(shadow, (int)(p / LAYER_SIZE), (int)(p % LAYER_SIZE), master[p]);
}

// sum of w in a fixed order (one block): out[0] = sum, out[2] = 1 / sum (0 if the sum is not
// positive and finite); the normalised loss is folded by dmc_flow_loss_kernel after the pass
__global__ void __launch_bounds__(256) dmc_flow_sums_kernel(const float* w, int64_t n, double* out) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) acc += (double)w[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
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
template <int D>
static hipError_t launch_sample_d(const FlowSampleArgs& a, int n_cu, hipStream_t st) {
    const int smem = flow_fwd_lds_bytes<D>();
    hipError_t e = hipFuncSetAttribute((const void*)dmc_flow_sample_kernel<D>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, smem);
    if (e != hipSuccess) return e;
    const int64_t want = (a.n + 255) / 256;
    const int grid = (int)(want < (int64_t)n_cu ? want : (int64_t)n_cu);
    hipLaunchKernelGGL(dmc_flow_sample_kernel<D>, dim3(grid), dim3(256), smem, st, a);
    return hipGetLastError();
}

int flow_sample_lds_bytes(int dim) {
    switch (dim) {
        case 3: return flow_fwd_lds_bytes<3>();
        case 7: return flow_fwd_lds_bytes<7>();
        case 11: return flow_fwd_lds_bytes<11>();
        case 15: return flow_fwd_lds_bytes<15>();
        case 19: return flow_fwd_lds_bytes<19>();
        case 23: return flow_fwd_lds_bytes<23>();
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

hipError_t launch_flow_inverse(const FlowTrainArgs& a, int nblk, hipStream_t st) {
    hipError_t e = hipFuncSetAttribute((const void*)dmc_flow_inverse_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, TRAIN_LDS);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(dmc_flow_inverse_kernel, dim3(nblk), dim3(256), TRAIN_LDS, st, a);
    return hipGetLastError();
}

hipError_t launch_flow_backward(const FlowTrainArgs& a, int nblk, int layer, int wg_chunk, int wg_blocks,
                                float* partial_layer, hipStream_t st) {
    hipError_t e = hipFuncSetAttribute((const void*)dmc_flow_bwd_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       TRAIN_LDS);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(dmc_flow_bwd_kernel, dim3(nblk), dim3(256), TRAIN_LDS, st, a, layer);
    hipLaunchKernelGGL(dmc_flow_wgrad_kernel, dim3(wg_blocks), dim3(256), 0, st, a, wg_chunk, partial_layer);
    return hipGetLastError();
}

hipError_t launch_flow_sums(const float* w, int64_t n, double* out, hipStream_t st) {
    hipLaunchKernelGGL(dmc_flow_sums_kernel, dim3(1), dim3(256), 0, st, w, n, out);
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

hipError_t launch_flow_mix(float* jac, const float* lq, int64_t n, float alpha, hipStream_t st) {
    const int64_t want = (n + 255) / 256;
    hipLaunchKernelGGL(dmc_flow_mix_kernel, dim3((unsigned)(want < 4096 ? want : 4096)), dim3(256), 0, st, jac, lq, n,
                       alpha);
    return hipGetLastError();
}

hipError_t launch_flow_shadow(const float* master, __bf16* shadow, int n_layers, int n_cu, hipStream_t st) {
    hipLaunchKernelGGL(dmc_flow_shadow_kernel, dim3(n_cu * 4), dim3(256), 0, st, master, shadow, n_layers);
    return hipGetLastError();
}

}  // namespace dmc
