// Neural spline flow kernels (Appendix A): rational-quadratic spline couplings on [0, 1] with a residual
// conditioner, uniform base.  One lane carries one sample through every layer, layer by layer.  In the
// sampling and inverse passes the 32 x 32 hidden layer and the spline-parameter layer run on the FP32
// matrix cores over the wave's 64 samples, handed back lane by lane; the first layer and the reverse
// sweep stay on the VALU with their weights, the same for every lane, in scalar registers.  The weight
// gradients, sums over samples of outer products, run on the matrix cores as well.  FP32 throughout.
//   dmc_nsf_sample_kernel     Philox z -> couplings -> u' -> VEGAS map -> physical map, mixture weight
//   dmc_nsf_inverse_kernel    u' -> z by the inverse couplings: log q(u'), optionally J_V(u'), every z_l, the
//                             base point and the flow's own weight
//   dmc_nsf_walk_kernel       the random-walk move of base points
//   dmc_nsf_backward_kernel   one layer of the reverse sweep of the weighted forward KL
//   dmc_nsf_outer_kernel      sums over samples of outer products (the weight gradients) on the FP32 matrix cores
#include <hip/hip_runtime.h>

#include <cstdint>

#include "nsf.hpp"

namespace dmc {

namespace {

constexpr float MINV = 1e-3f;  // minimum bin width, height and interior derivative

__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
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

// the uniform sampler's draw: coordinate d of sample i from counter (i lo, i hi, d / 4, 0), word d % 4
template <class V>
__device__ __forceinline__ void philox_point(uint64_t seed, uint64_t i, int D, V u) {
    for (int q = 0; q < (D + 3) / 4; ++q) {
        uint32_t c[4] = {(uint32_t)i, (uint32_t)(i >> 32), (uint32_t)q, 0u};
        philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
        for (int w = 0; w < 4 && 4 * q + w < D; ++w) u[4 * q + w] = ((float)(c[w] >> 8) + 0.5f) * 0x1p-24f;
    }
}

// A lane's D coordinates in LDS, one column per thread of a 256-thread block: indexed by the coupling
// masks, which are known only at run time, the coordinates would otherwise live in scratch memory
constexpr int NSF_BLOCK = 256;
struct LdsCol {
    float* p;
    __device__ __forceinline__ float& operator[](int d) const { return p[d * NSF_BLOCK]; }
};

// Elementary functions of the spline.  With Fast, e^x comes from the hardware 2^x of x log2(e), whose
// rounding gives a relative error of about 6e-8 |x| (the arguments are softmax logits less their maximum
// and -|t|, a few tens at most); otherwise from the accurate library exp.  Reciprocals come from the
// hardware reciprocal (1 ulp) wherever the divisor is bounded away from zero and overflow.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
// softplus(t) = max(t, 0) + log1p(e^-|t|), with log1p(e) = log(u) e / (u - 1) for u = 1 + e rounded
// (Goldberg's formula: exact to a few ulp from an accurate log)
template <bool Fast>
__device__ __forceinline__ float softplusf(float t) {
    const float e = Fast ? __expf(-fabsf(t)) : expf(-fabsf(t)), u = 1.0f + e;
    const float lp = u == 1.0f ? e : logf(u) * (e * rcp(u - 1.0f));
    return lp + fmaxf(t, 0.0f);
}
__device__ __forceinline__ float sigmoidf_(float t) { return 1.0f / (1.0f + expf(-t)); }

// Softmax probabilities of the widths (sw) and heights (sh) and the knot derivatives d[0..K] of one
// coordinate's spline from its NP parameters
template <bool Fast>
__device__ __forceinline__ void spline_shape(const float* th, float* sw, float* sh, float* d) {
    float mw = th[0], mh = th[NSF_K];
#pragma unroll
    for (int i = 1; i < NSF_K; ++i) {
        mw = fmaxf(mw, th[i]);
        mh = fmaxf(mh, th[NSF_K + i]);
    }
    float zw = 0.0f, zh = 0.0f;
#pragma unroll
    for (int i = 0; i < NSF_K; ++i) {
        sw[i] = Fast ? __expf(th[i] - mw) : expf(th[i] - mw);
        sh[i] = Fast ? __expf(th[NSF_K + i] - mh) : expf(th[NSF_K + i] - mh);
        zw += sw[i];
        zh += sh[i];
    }
    const float cw = Fast ? rcp(zw) : 1.0f / zw, ch = Fast ? rcp(zh) : 1.0f / zh;
#pragma unroll
    for (int i = 0; i < NSF_K; ++i) {
        sw[i] *= cw;
        sh[i] *= ch;
    }
    d[0] = 1.0f;
    d[NSF_K] = 1.0f;
#pragma unroll
    for (int i = 1; i < NSF_K; ++i) d[i] = MINV + softplusf<Fast>(th[2 * NSF_K + i - 1]);
}

// The bin holding v and its knots.  Knot i + 1 is knot i plus m + (1 - K m) times the softmax probability,
// the last knot is 1 on both axes; the bin is the last one whose left knot (on x, or on y for the inverse)
// is <= v.  An unrolled scan with selects: every array index is a constant, so nothing leaves registers.
struct Bin {
    float xk, yk, W, H, d0, d1;
    int k;
};

__device__ __forceinline__ Bin find_bin(const float* sw, const float* sh, const float* d, float v, bool on_y) {
    const float scale = 1.0f - NSF_K * MINV;
    Bin b;
    float cx = 0.0f, cy = 0.0f;
#pragma unroll
    for (int i = 0; i < NSF_K; ++i) {
        const float nx = i == NSF_K - 1 ? 1.0f : cx + (MINV + scale * sw[i]);
        const float ny = i == NSF_K - 1 ? 1.0f : cy + (MINV + scale * sh[i]);
        if (i == 0 || (on_y ? cy : cx) <= v) {
            b.xk = cx;
            b.yk = cy;
            b.W = nx - cx;
            b.H = ny - cy;
            b.k = i;
        }
        cx = nx;
        cy = ny;
    }
    // the knot derivatives by a second pass of selects on the bin index (selecting them in the scan above
    // lets the compiler turn d into a scratch array indexed at run time)
    b.d0 = d[0];
    b.d1 = d[1];
#pragma unroll
    for (int i = 1; i < NSF_K; ++i) {
        b.d0 = b.k == i ? d[i] : b.d0;
        b.d1 = b.k == i ? d[i + 1] : b.d1;
    }
    return b;
}

// forward spline: v -> y, returns log dy/dx
__device__ __forceinline__ float spline_fwd(const float* th, float& v) {
    float sw[NSF_K], sh[NSF_K], d[NSF_K + 1];
    spline_shape<true>(th, sw, sh, d);
    const Bin b = find_bin(sw, sh, d, v, false);
    const float rW = rcp(b.W), s = b.H * rW;
    const float xi = fminf(fmaxf((v - b.xk) * rW, 0.0f), 1.0f), t = xi * (1.0f - xi);
    const float den = s + (b.d1 + b.d0 - 2.0f * s) * t, rden = rcp(den);
    v = b.yk + b.H * (s * xi * xi + b.d0 * t) * rden;
    const float num = b.d1 * xi * xi + 2.0f * s * t + b.d0 * (1.0f - xi) * (1.0f - xi);
    // log(s^2 num / den^2): s, num and den lie within [1e-3, 1e3] or so, far from FP32's limits
    return logf(s * s * num * (rden * rden));
}

// inverse spline: v (an output) -> x, returns log dy/dx at x
template <bool Fast>
__device__ __forceinline__ float spline_inv(const float* th, float& v) {
    float sw[NSF_K], sh[NSF_K], d[NSF_K + 1];
    spline_shape<Fast>(th, sw, sh, d);
    const Bin b = find_bin(sw, sh, d, v, true);
    const float W = b.W, H = b.H, s = H * rcp(W);
    const float dy = v - b.yk, g = b.d1 + b.d0 - 2.0f * s;
    const float qa = H * (s - b.d0) + dy * g, qb = H * b.d0 - dy * g, qc = -s * dy;
    const float sq = sqrtf(fmaxf(qb * qb - 4.0f * qa * qc, 0.0f));
    // the root of the quadratic in its stable form; -qb - sq < 0 unless dy = 0, where 0 / 0 is clamped to 0
    const float xi = fminf(fmaxf(2.0f * qc / (-qb - sq), 0.0f), 1.0f), t = xi * (1.0f - xi);
    v = b.xk + xi * W;
    const float den = s + g * t, rden = rcp(den);
    const float num = b.d1 * xi * xi + 2.0f * s * t + b.d0 * (1.0f - xi) * (1.0f - xi);
    return logf(s * s * num * (rden * rden));
}

// Reverse sweep of phi = gx x + gl log(dy/dx) through the inverse spline at output v: returns
// d phi / d v and writes d phi / d theta (NP values).
__device__ __forceinline__ float spline_inv_adjoint(const float* th, float v, float gx, float gl, float* gth) {
    float sw[NSF_K], sh[NSF_K], d[NSF_K + 1];
    spline_shape<false>(th, sw, sh, d);
    const Bin bn = find_bin(sw, sh, d, v, true);
    const int k = bn.k;
    const float W = bn.W, H = bn.H, s = H / W;
    const float d0 = bn.d0, d1 = bn.d1;
    const float dy = v - bn.yk, g = d1 + d0 - 2.0f * s;
    const float a = H * (s - d0) + dy * g, b = H * d0 - dy * g, c = -s * dy;
    const float sq = sqrtf(fmaxf(b * b - 4.0f * a * c, 0.0f));
    const float q = -b - sq;
    const float xi = 2.0f * c / q, t = xi * (1.0f - xi);
    const float den = s + g * t;
    const float num = d1 * xi * xi + 2.0f * s * t + d0 * (1.0f - xi) * (1.0f - xi);
    // adjoints
    float b_xk = gx, b_xi = gx * W, b_W = gx * xi;
    float b_s = 2.0f * gl / s;
    const float b_num = gl / num, b_den = -2.0f * gl / den;
    b_s += b_den;
    float b_g = b_den * t, b_t = b_den * g;
    float b_d1 = b_num * xi * xi, b_d0 = b_num * (1.0f - xi) * (1.0f - xi);
    b_xi += b_num * (2.0f * d1 * xi - 2.0f * d0 * (1.0f - xi));
    b_s += b_num * 2.0f * t;
    b_t += b_num * 2.0f * s;
    b_xi += b_t * (1.0f - 2.0f * xi);
    float b_c = 2.0f * b_xi / q;
    const float b_q = -b_xi * xi / q;
    float b_b = -b_q;
    const float b_sq = -b_q;
    const float b_disc = sq > 0.0f ? b_sq / (2.0f * sq) : 0.0f;
    b_b += b_disc * 2.0f * b;
    const float b_a = -4.0f * c * b_disc;
    b_c += -4.0f * a * b_disc;
    b_s += -dy * b_c;
    float b_dy = -s * b_c;
    float b_H = b_b * d0;
    b_d0 += b_b * H;
    b_dy += -b_b * g;
    b_g += -b_b * dy;
    b_H += b_a * (s - d0);
    b_s += b_a * H;
    b_d0 += -b_a * H;
    b_dy += b_a * g;
    b_g += b_a * dy;
    b_d1 += b_g;
    b_d0 += b_g;
    b_s += -2.0f * b_g;
    const float b_v = b_dy, b_yk = -b_dy;
    b_H += b_s / W;
    b_W += -b_s * H / (W * W);
    // knots: x_k = sum_{i<k} w_i, W = w_k; likewise y, H
    float bw[NSF_K], bh[NSF_K];
#pragma unroll
    for (int i = 0; i < NSF_K; ++i) {
        bw[i] = i < k ? b_xk : (i == k ? b_W : 0.0f);
        bh[i] = i < k ? b_yk : (i == k ? b_H : 0.0f);
    }
    // w = m + (1 - K m) softmax(theta_w): dtheta_i = (1 - K m) sw_i (bw_i - sum_j sw_j bw_j)
    float pw = 0.0f, ph = 0.0f;
#pragma unroll
    for (int i = 0; i < NSF_K; ++i) {
        pw += sw[i] * bw[i];
        ph += sh[i] * bh[i];
    }
    const float scale = 1.0f - NSF_K * MINV;
#pragma unroll
    for (int i = 0; i < NSF_K; ++i) {
        gth[i] = scale * sw[i] * (bw[i] - pw);
        gth[NSF_K + i] = scale * sh[i] * (bh[i] - ph);
    }
    // interior derivatives d_i (i = 1..K-1) = m + softplus(theta[2K + i - 1]): d_k takes b_d0, d_{k+1} b_d1
#pragma unroll
    for (int i = 1; i < NSF_K; ++i) {
        const float bd = i == k ? b_d0 : (i == k + 1 ? b_d1 : 0.0f);
        gth[2 * NSF_K + i - 1] = bd * sigmoidf_(th[2 * NSF_K + i - 1]);
    }
    return b_v;
}

// parameters are read through the constant address space: the addresses are uniform across a wave, so the
// compiler loads them into scalar registers (no LDS traffic per multiply-add)
typedef const __attribute__((address_space(4))) float* cfloat_p;
struct Layer {
    cfloat_p W1, b1, W2, b2, W3, b3;
    int dA, dB, P;
};

// views of layer l's parameters, read in place
__device__ __forceinline__ Layer layer_view(const float* params, int off, int dA, int dB) {
    const int P = NSF_NP * dB;
    Layer L;
    L.dA = dA;
    L.dB = dB;
    L.P = P;
    L.W1 = (cfloat_p)(params + off);
    L.b1 = L.W1 + NSF_H * dA;
    L.W2 = L.b1 + NSF_H;
    L.b2 = L.W2 + NSF_H * NSF_H;
    L.W3 = L.b2 + NSF_H;
    L.b3 = L.W3 + P * NSF_H;
    return L;
}

// a1 = relu(W1 zA + b1), a2 = relu(W2 a1 + b2) + a1; pre-activation signs in m1, m2
__device__ __forceinline__ void conditioner(const Layer& L, const float* zA, float* a1, float* a2, uint32_t& m1,
                                            uint32_t& m2) {
    m1 = m2 = 0u;
    for (int h = 0; h < NSF_H; ++h) {
        float p = L.b1[h];
        for (int i = 0; i < L.dA; ++i) p = __builtin_fmaf(L.W1[h * L.dA + i], zA[i], p);
        a1[h] = fmaxf(p, 0.0f);
        m1 |= (p > 0.0f ? 1u : 0u) << h;
    }
    for (int h = 0; h < NSF_H; ++h) {
        float p = L.b2[h];
        for (int i = 0; i < NSF_H; ++i) p = __builtin_fmaf(L.W2[h * NSF_H + i], a1[i], p);
        a2[h] = fmaxf(p, 0.0f) + a1[h];
        m2 |= (p > 0.0f ? 1u : 0u) << h;
    }
}

// the NP parameters of transformed coordinate j, two rows of W3 at a time
__device__ __forceinline__ void spline_params(const Layer& L, const float* a2, int j, float* th) {
    for (int r = 0; r + 1 < NSF_NP; r += 2) {
        const int row = j * NSF_NP + r;
        float p0 = L.b3[row], p1 = L.b3[row + 1];
        for (int h = 0; h < NSF_H; ++h) {
            p0 = __builtin_fmaf(L.W3[row * NSF_H + h], a2[h], p0);
            p1 = __builtin_fmaf(L.W3[(row + 1) * NSF_H + h], a2[h], p1);
        }
        th[r] = p0;
        th[r + 1] = p1;
    }
    if (NSF_NP % 2) {
        const int row = j * NSF_NP + NSF_NP - 1;
        float p = L.b3[row];
        for (int h = 0; h < NSF_H; ++h) p = __builtin_fmaf(L.W3[row * NSF_H + h], a2[h], p);
        th[NSF_NP - 1] = p;
    }
}

typedef float f32x16 __attribute__((ext_vector_type(16)));

// lanes 32..63 of x trade places with lanes 0..31 of y
__device__ __forceinline__ void swap32(float& x, float& y) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
    x = __uint_as_float(r[0]);
    y = __uint_as_float(r[1]);
}

// Matrix-core products of the conditioner for the wave's 64 samples (lane = sample), y[r] = sum_h W[row0 + r][h]
// x[h] for r < 32, on FP32 MFMA 32x32x2: samples 0..31 form one output tile, samples 32..63 the other.  In
// MFMA step t the two K slots carry h = t (lanes 0..31) and h = 16 + t (lanes 32..63).  mfma_operands turns a
// lane's own x into those B operands; rows_mfma takes a lane's 16 weights of row row0 + lane % 32 and hands
// every lane the 32 outputs of its own sample.  Every lane of the wave must take part.
__device__ __forceinline__ void mfma_operands(const float* x, float* b0, float* b1) {
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        b0[t] = x[t];
        b1[t] = x[16 + t];
        swap32(b0[t], b1[t]);
    }
}

// a lane's 16 weights of row row0 + lane % 32 (zero past the last row)
__device__ __forceinline__ void load_rows(const float* W, int rows, int row0, float* w) {
    const int lane = threadIdx.x & 63, m = lane & 31, hh = lane >> 5;
    const int row = row0 + m;
    const bool ok = row < rows;
    const float* wr = W + (int64_t)(ok ? row : 0) * NSF_H + 16 * hh;
#pragma unroll
    for (int t = 0; t < 16; ++t) w[t] = ok ? wr[t] : 0.0f;
}

__device__ __forceinline__ void rows_mfma(const float* w, const float* b0, const float* b1, float* y) {
    f32x16 c0, c1;
#pragma unroll
    for (int v = 0; v < 16; ++v) c0[v] = c1[v] = 0.0f;
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(w[t], b0[t], c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(w[t], b1[t], c1, 0, 0, 0);
    }
    // register v of a tile holds row 8 (v / 4) + 4 (lane / 32) + v % 4 for sample lane % 32 of the tile
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        float p = c0[v], q = c1[v];
        swap32(p, q);
        y[8 * (v / 4) + v % 4] = p;
        y[8 * (v / 4) + 4 + v % 4] = q;
    }
}

// a1 = relu(W1 zA + b1) on the VALU (zA: the coordinates z[aidx[i]], i < dA), a2 = relu(W2 a1 + b2) + a1 on the
// matrix cores; b0, b1 receive a2 as B operands for the spline-parameter rows
template <class V>
__device__ __forceinline__ void conditioner_mfma(const Layer& L, const float* Wg, V z, const int* aidx, float* b0,
                                                 float* b1) {
    // the first layer takes the kept coordinates one at a time (the same order of sums as row by row), so
    // that no array is indexed at run time
    float a1[NSF_H], pre[NSF_H];
#pragma unroll
    for (int h = 0; h < NSF_H; ++h) a1[h] = L.b1[h];
    for (int i = 0; i < L.dA; ++i) {
        const float zi = z[aidx[i]];
#pragma unroll
        for (int h = 0; h < NSF_H; ++h) a1[h] = __builtin_fmaf(L.W1[h * L.dA + i], zi, a1[h]);
    }
#pragma unroll
    for (int h = 0; h < NSF_H; ++h) a1[h] = fmaxf(a1[h], 0.0f);
    mfma_operands(a1, b0, b1);
    float w[16];
    load_rows(Wg + NSF_H * L.dA + NSF_H, NSF_H, 0, w);
    rows_mfma(w, b0, b1, pre);
    float a2[NSF_H];
#pragma unroll
    for (int h = 0; h < NSF_H; ++h) a2[h] = fmaxf(pre[h] + L.b2[h], 0.0f) + a1[h];
    mfma_operands(a2, b0, b1);
}

// the spline-parameter rows: W3 of the layer (its P rows start at row j NP for coordinate j)
__device__ __forceinline__ const float* w3_rows(const Layer& L, const float* Wg) {
    return Wg + NSF_H * L.dA + NSF_H + NSF_H * NSF_H + NSF_H;
}

// the NP parameters of transformed coordinate j from the B operands of a2 and the lane's W3 weights w (as
// load_rows gives them for row0 = j NP); w then receives those of coordinate j + 1, so that their loads
// overlap the spline of coordinate j
__device__ __forceinline__ void spline_params_mfma(const Layer& L, const float* W3, const float* b0, const float* b1,
                                                   int j, float* w, float* th) {
    float t[32];
    rows_mfma(w, b0, b1, t);
    if (j + 1 < L.dB) load_rows(W3, L.P, (j + 1) * NSF_NP, w);
#pragma unroll
    for (int r = 0; r < NSF_NP; ++r) th[r] = t[r] + L.b3[j * NSF_NP + r];
}

}  // namespace

// flow share: Philox z -> every coupling forward -> u'; VEGAS map, physical map, mixture weight
__global__ void __launch_bounds__(NSF_BLOCK, 4) dmc_nsf_sample_kernel(NsfArgs a) {
    __shared__ float zl[NSF_MAXD * NSF_BLOCK];
    const int D = a.dim, N = (D + 1) / 4;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < a.n; base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = base + threadIdx.x;
        const bool valid = s < a.n;
        const LdsCol z{zl + threadIdx.x};
        if (a.z_in) {
            for (int d = 0; d < D; ++d) z[d] = a.z_in[(int64_t)d * a.ld_z + (valid ? s : 0)];
        } else {
            philox_point(a.seed, a.first + (uint64_t)(valid ? s : 0), D, z);
        }
        float lq = 0.0f;
        for (int l = 0; l < a.n_layers; ++l) {
            const Layer L = layer_view(a.params, a.offs[l], a.dA[l], D - a.dA[l]);
            const float* Wg = a.params + a.offs[l];
            float b0[16], b1[16], th[NSF_NP];
            conditioner_mfma(L, Wg, z, a.aidx + l * NSF_MAXD, b0, b1);
            const float* W3 = w3_rows(L, Wg);
            float w[16];
            load_rows(W3, L.P, 0, w);
            for (int j = 0; j < L.dB; ++j) {
                spline_params_mfma(L, W3, b0, b1, j, w, th);
                const int col = a.bidx[l * NSF_MAXD + j];
                float v = z[col];
                lq -= spline_fwd(th, v);
                z[col] = v;
            }
        }
        if (!valid) continue;
        // the grid map replaces each u' by y in the lane's LDS column
        const LdsCol& y = z;
        float J = 1.0f, jv = 1.0f;
        for (int d = 0; d < D; ++d) {
            const float up = z[d];
            if (a.u_out) a.u_out[(int64_t)d * a.ld + s] = up;
            const float ub = up * (float)a.n_bins;
            const int bin = (int)fminf(fmaxf(ub, 0.0f), (float)(a.n_bins - 1));
            const float fr = ub - (float)bin;
            const float lo = a.edges[d * (a.n_bins + 1) + bin];
            const float hi = a.edges[d * (a.n_bins + 1) + bin + 1];
            y[d] = __builtin_fmaf(fr, hi - lo, lo);
            jv *= (float)a.n_bins * (hi - lo);
        }
        for (int q = 0; q < N; ++q) {
            const float r = a.qmax * y[3 * q];
            const float ct = __builtin_fmaf(2.0f, y[3 * q + 1], -1.0f);
            const float st = sqrtf(fmaxf(0.0f, __builtin_fmaf(-ct, ct, 1.0f)));
            float sp, cp;
            sincospif(2.0f * y[3 * q + 2], &sp, &cp);
            a.x[(int64_t)(3 * q) * a.ld + s] = r * st * cp;
            a.x[(int64_t)(3 * q + 1) * a.ld + s] = r * st * sp;
            a.x[(int64_t)(3 * q + 2) * a.ld + s] = r * ct;
            J *= a.jl * r * r;
        }
        for (int jt = 1; jt < N; ++jt) a.x[(int64_t)(3 * N + jt - 1) * a.ld + s] = a.beta * y[3 * N + jt - 1];
        a.jac[s] = J * jv * a.jt / __builtin_fmaf(a.mix_f, expf(lq), __builtin_fmaf(a.mix_u, jv, a.mix_g));
        if (a.jf_out) a.jf_out[s] = J * jv * a.jt / expf(lq);
        if (a.lq_out) a.lq_out[s] = lq;
    }
}

// u' -> z by the inverse couplings (last layer first); log q(u') = -sum of the layers' log dy/dx.  The pass
// that feeds training (Fast = false) takes the accurate e^x: the weight gradients of a peaked flow magnify
// its rounding.
template <bool Fast>
__global__ void __launch_bounds__(NSF_BLOCK, 4) dmc_nsf_inverse_kernel(NsfArgs a) {
    __shared__ float zl[NSF_MAXD * NSF_BLOCK];
    const int D = a.dim, L_ = a.n_layers;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < a.n; base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = base + threadIdx.x;
        const bool valid = s < a.n;
        const int64_t sc = valid ? s : 0;
        const LdsCol z{zl + threadIdx.x};
        if (a.u_in) {
            for (int d = 0; d < D; ++d) z[d] = a.u_in[(int64_t)d * a.ld + sc];
        } else {
            philox_point(a.seed, a.first + (uint64_t)sc, D, z);
        }
        float jphys = 0.0f;
        if (valid) {
            if (a.u_out && !a.u_in)
                for (int d = 0; d < D; ++d) a.u_out[(int64_t)d * a.ld + s] = z[d];
            if (a.jv_out || a.jf_out) {
                // the grid's Jacobian, and with jf_out the physical map's (r = qmax y per loop) as the
                // sampling pass forms them
                float jv = 1.0f, J = 1.0f;
                for (int d = 0; d < D; ++d) {
                    const float ub = z[d] * (float)a.n_bins;
                    const int bin = (int)fminf(fmaxf(ub, 0.0f), (float)(a.n_bins - 1));
                    const float fr = ub - (float)bin;
                    const float lo = a.edges[d * (a.n_bins + 1) + bin];
                    const float hi = a.edges[d * (a.n_bins + 1) + bin + 1];
                    if (d % 3 == 0 && d < 3 * ((D + 1) / 4)) {
                        const float r = a.qmax * __builtin_fmaf(fr, hi - lo, lo);
                        J *= a.jl * r * r;
                    }
                    jv *= (float)a.n_bins * (hi - lo);
                }
                if (a.jv_out) a.jv_out[s] = jv;
                jphys = J * jv * a.jt;
            }
            if (a.zs)
                for (int d = 0; d < D; ++d) a.zs[((int64_t)L_ * D + d) * a.n + s] = z[d];
        }
        float lq = 0.0f;
        for (int l = L_ - 1; l >= 0; --l) {
            const Layer L = layer_view(a.params, a.offs[l], a.dA[l], D - a.dA[l]);
            const float* Wg = a.params + a.offs[l];
            float b0[16], b1[16], th[NSF_NP];
            conditioner_mfma(L, Wg, z, a.aidx + l * NSF_MAXD, b0, b1);
            const float* W3 = w3_rows(L, Wg);
            float w[16];
            load_rows(W3, L.P, 0, w);
            for (int j = 0; j < L.dB; ++j) {
                spline_params_mfma(L, W3, b0, b1, j, w, th);
                const int col = a.bidx[l * NSF_MAXD + j];
                float v = z[col];
                lq -= spline_inv<Fast>(th, v);
                z[col] = v;
            }
            if (valid && a.zs)
                for (int d = 0; d < D; ++d) a.zs[((int64_t)l * D + d) * a.n + s] = z[d];
        }
        if (valid && a.lq_out) a.lq_out[s] = lq;
        if (valid && a.jf_out) a.jf_out[s] = jphys / expf(lq);
        if (valid && a.z0_out)
            for (int d = 0; d < D; ++d) a.z0_out[(int64_t)d * a.ld_z + s] = z[d];
    }
}

// Base-space random walk (Sec. IV's optional proposal): z <- z + sigma xi, wrapped onto [0, 1).  Pair j of
// coordinates (2j, 2j + 1) of point i takes the Philox words of counter (i lo, i hi, j, 1), key seed: with
// u_k = ((w_k >> 8) + 1/2) 2^-24 and r = sqrt(-2 log u_0), xi = r cos(2 pi u_1), r sin(2 pi u_1) (Box-Muller).
__global__ void __launch_bounds__(256) dmc_nsf_walk_kernel(float* z, int D, int64_t n, int64_t ld, float sigma,
                                                            uint64_t seed, uint64_t first) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t g = first + (uint64_t)i;
        for (int j = 0; 2 * j < D; ++j) {
            uint32_t c[4] = {(uint32_t)g, (uint32_t)(g >> 32), (uint32_t)j, 1u};
            philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
            const float u0 = ((float)(c[0] >> 8) + 0.5f) * 0x1p-24f, u1 = ((float)(c[1] >> 8) + 0.5f) * 0x1p-24f;
            const float r = sqrtf(-2.0f * logf(u0));
            float sn, cs;
            sincospif(2.0f * u1, &sn, &cs);
            for (int k = 0; k < 2 && 2 * j + k < D; ++k) {
                float* p = z + (int64_t)(2 * j + k) * ld + i;
                float v = __builtin_fmaf(sigma, r * (k ? sn : cs), *p);
                v -= floorf(v);
                *p = v < 1.0f ? v : 0.0f;  // a tiny negative step rounds v - floor(v) up to 1
            }
        }
    }
}

// Layer reverse step: adj holds dL/dz_{l-1} (the layer's input side) on entry and dL/dz_l on exit
__global__ void __launch_bounds__(256) dmc_nsf_backward_kernel(NsfBackArgs a) {
    const Layer L = layer_view(a.params, a.off, a.dA, a.dB);
    const double inv = *a.inv_wsum;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < a.n; s += (int64_t)gridDim.x * blockDim.x) {
        const float wn = (float)((double)a.w[s] * inv);
        float zA[NSF_MAXD], a1[NSF_H], a2[NSF_H], da2[NSF_H], th[NSF_NP], gth[NSF_NP];
        uint32_t m1, m2;
        for (int i = 0; i < a.dA; ++i) zA[i] = a.z[(int64_t)a.aidx[i] * a.n + s];
        conditioner(L, zA, a1, a2, m1, m2);
        for (int h = 0; h < NSF_H; ++h) da2[h] = 0.0f;
        for (int j = 0; j < a.dB; ++j) {
            spline_params(L, a2, j, th);
            const int col = a.bidx[j];
            const float v = a.z[(int64_t)col * a.n + s];
            const float gx = a.adj[(int64_t)col * a.n + s];
            const float gv = spline_inv_adjoint(th, v, gx, wn, gth);
            a.adj[(int64_t)col * a.n + s] = gv;
            for (int r = 0; r < NSF_NP; ++r) {
                const int row = j * NSF_NP + r;
                a.d_theta[(int64_t)row * a.n + s] = gth[r];
                for (int h = 0; h < NSF_H; ++h) da2[h] = __builtin_fmaf(L.W3[row * NSF_H + h], gth[r], da2[h]);
            }
        }
        // a2 = relu(pre2) + a1, a1 = relu(pre1)
        float dp2[NSF_H], da1[NSF_H];
        for (int h = 0; h < NSF_H; ++h) {
            dp2[h] = (m2 >> h) & 1u ? da2[h] : 0.0f;
            da1[h] = da2[h];
        }
        for (int i = 0; i < NSF_H; ++i) {
            float acc = da1[i];
            for (int h = 0; h < NSF_H; ++h) acc = __builtin_fmaf(L.W2[h * NSF_H + i], dp2[h], acc);
            da1[i] = acc;
        }
        for (int h = 0; h < NSF_H; ++h) {
            const float dp1 = (m1 >> h) & 1u ? da1[h] : 0.0f;
            a.a2[(int64_t)h * a.n + s] = a2[h];
            a.d_pre2[(int64_t)h * a.n + s] = dp2[h];
            a.a1[(int64_t)h * a.n + s] = a1[h];
            a.d_pre1[(int64_t)h * a.n + s] = dp1;
            da1[h] = dp1;
        }
        for (int i = 0; i < a.dA; ++i) {
            float acc = 0.0f;
            for (int h = 0; h < NSF_H; ++h) acc = __builtin_fmaf(L.W1[h * a.dA + i], da1[h], acc);
            const int col = a.aidx[i];
            a.adj[(int64_t)col * a.n + s] += acc;
            a.zA[(int64_t)i * a.n + s] = zA[i];
        }
    }
}

// Sums over samples of outer products on the matrix cores (FP32 MFMA 32x32x2), C[i][j] = sum_n A[i][n] B[j][n]
// with rowsB <= 32.  A block takes one chunk of OUTER_CHUNK samples and up to OUTER_TILES tiles of 32 rows of
// A against every row of B.  Each wave sweeps groups of 32 samples of the chunk: lane half h feeds samples
// 16 h .. 16 h + 15 of the group into the two K slots of 16 successive MFMAs, so a lane reads 16 consecutive
// values of one row of A and of one row of B.  The row sums of A (the bias gradient) ride along on the VALU.
// The waves' tiles are added in LDS in wave order, and the chunks in chunk order by the fold: deterministic.
constexpr int OUTER_CHUNK = 512;
constexpr int OUTER_TILES = 4;
constexpr int OUTER_WAVES = 4;
__device__ __forceinline__ void load16(const float* M, int row, int rows, int64_t s0, int64_t n1, int64_t n, bool vec,
                                       float* v) {
    if (vec && row < rows && s0 + 16 <= n1) {
        const float4* q = reinterpret_cast<const float4*>(M + (int64_t)row * n + s0);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float4 t = q[k];
            v[4 * k] = t.x;
            v[4 * k + 1] = t.y;
            v[4 * k + 2] = t.z;
            v[4 * k + 3] = t.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = (row < rows && s0 + k < n1) ? M[(int64_t)row * n + s0 + k] : 0.0f;
    }
}

__global__ void __launch_bounds__(64 * OUTER_WAVES) dmc_nsf_outer_kernel(const float* A, int rowsA, const float* B,
                                                                          int rowsB, int64_t n, float* partial) {
    __shared__ float red[OUTER_WAVES][32 * 32 + 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, h = lane >> 5, r = lane & 31;
    const int t0 = blockIdx.x * OUTER_TILES, tiles = (rowsA + 31) / 32;
    const int nt = tiles - t0 < OUTER_TILES ? tiles - t0 : OUTER_TILES;
    const int64_t c = blockIdx.y, n0 = c * OUTER_CHUNK, n1 = n0 + OUTER_CHUNK < n ? n0 + OUTER_CHUNK : n;
    // 16-byte loads when every row starts 16-byte aligned (chunk starts are multiples of 16 samples)
    const bool vec = (n & 3) == 0 && ((uintptr_t)A & 15) == 0 && ((uintptr_t)B & 15) == 0;
    f32x16 acc[OUTER_TILES];
    float bias[OUTER_TILES];
#pragma unroll
    for (int q = 0; q < OUTER_TILES; ++q) {
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[q][v] = 0.0f;
        bias[q] = 0.0f;
    }
    for (int64_t g = n0 + 32 * wave; g < n1; g += 32 * OUTER_WAVES) {
        const int64_t s0 = g + 16 * h;
        float bv[16];
        load16(B, r, rowsB, s0, n1, n, vec, bv);
#pragma unroll
        for (int q = 0; q < OUTER_TILES; ++q) {
            if (q < nt) {
                float av[16];
                load16(A, (t0 + q) * 32 + r, rowsA, s0, n1, n, vec, av);
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[k], bv[k], acc[q], 0, 0, 0);
                    bias[q] += av[k];
                }
            }
        }
    }
    const int cols = rowsB + 1;
#pragma unroll
    for (int q = 0; q < OUTER_TILES; ++q) {
        if (q >= nt) break;
        __syncthreads();
        // accumulator register v of lane (h, r): tile row 8 (v / 4) + 4 h + v % 4, column r
#pragma unroll
        for (int v = 0; v < 16; ++v) red[wave][(8 * (v / 4) + 4 * h + v % 4) * 32 + r] = acc[q][v];
        red[wave][1024 + lane] = bias[q];
        __syncthreads();
        for (int e = threadIdx.x; e < 32 * cols; e += 64 * OUTER_WAVES) {
            const int i = e / cols, j = e % cols, row = (t0 + q) * 32 + i;
            if (row >= rowsA) continue;
            float s = 0.0f;
            for (int w = 0; w < OUTER_WAVES; ++w)
                s += j < rowsB ? red[w][i * 32 + j] : red[w][1024 + i] + red[w][1024 + 32 + i];
            partial[(c * rowsA + row) * cols + j] = s;
        }
    }
}

// grad[i][j] = sum over chunks of partial[c][i][j]: a block of 1024 threads takes 64 outputs, its 16 waves
// take every 16th chunk, and the 16 sums are added in wave order
__global__ void __launch_bounds__(1024) dmc_nsf_outer_fold_kernel(const float* partial, int rowsA, int rowsB,
                                                                   int chunks, float* grad) {
    __shared__ float red[16][64];
    const int cols = rowsB + 1, total = rowsA * cols;
    const int o = threadIdx.x & 63, part = threadIdx.x >> 6;
    const int t = blockIdx.x * 64 + o;
    float s = 0.0f;
    if (t < total)
        for (int c = part; c < chunks; c += 16) s += partial[(int64_t)c * total + t];
    red[part][o] = s;
    __syncthreads();
    if (part != 0 || t >= total) return;
    float u = 0.0f;
    for (int p = 0; p < 16; ++p) u += red[p][o];
    const int i = t / cols, j = t % cols;
    // weights [rowsA][rowsB] then biases [rowsA]
    if (j < rowsB)
        grad[i * rowsB + j] = u;
    else
        grad[rowsA * rowsB + i] = u;
}

__global__ void __launch_bounds__(1024) dmc_nsf_loss_kernel(const float* w, const float* lq, int64_t n, double* out) {
    __shared__ double r0[1024], r1[1024];
    double s0 = 0.0, s1 = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) {
        const double wi = (double)w[i];
        const double li = (double)lq[i];
        if (wi > 0.0 && __builtin_isfinite(li)) {
            s0 += wi;
            s1 += wi * li;
        }
    }
    r0[threadIdx.x] = s0;
    r1[threadIdx.x] = s1;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            r0[threadIdx.x] += r0[threadIdx.x + o];
            r1[threadIdx.x] += r1[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = r0[0];
        out[1] = r1[0];
        out[2] = r0[0] > 0.0 ? 1.0 / r0[0] : 0.0;  // 1 / sum w
        out[3] = r0[0] > 0.0 ? -r1[0] / r0[0] : 0.0;  // the loss
    }
}

__global__ void __launch_bounds__(256) dmc_nsf_adam_kernel(float* p, float* m, float* v, const float* g, int64_t count,
                                                            float lr, float c1, float c2) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        if (!__builtin_isfinite(gi)) continue;
        const float mi = 0.9f * m[i] + 0.1f * gi;
        const float vi = 0.999f * v[i] + 0.001f * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + 1e-8f);
    }
}

static int grid_for(int64_t n, int n_cu) {
    const int64_t want = (n + 255) / 256;
    const int64_t cap = (int64_t)n_cu * 4;
    return (int)(want < cap ? (want > 0 ? want : 1) : cap);
}

hipError_t launch_nsf_sample(const NsfArgs& a, int n_cu, hipStream_t st) {
    hipLaunchKernelGGL(dmc_nsf_sample_kernel, dim3(grid_for(a.n, n_cu)), dim3(NSF_BLOCK), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_nsf_inverse(const NsfArgs& a, int n_cu, hipStream_t st) {
    if (a.zs)
        hipLaunchKernelGGL(dmc_nsf_inverse_kernel<false>, dim3(grid_for(a.n, n_cu)), dim3(NSF_BLOCK), 0, st, a);
    else
        hipLaunchKernelGGL(dmc_nsf_inverse_kernel<true>, dim3(grid_for(a.n, n_cu)), dim3(NSF_BLOCK), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_nsf_walk(float* z, int D, int64_t n, int64_t ld, float sigma, uint64_t seed, uint64_t first,
                           int n_cu, hipStream_t st) {
    hipLaunchKernelGGL(dmc_nsf_walk_kernel, dim3(grid_for(n, n_cu)), dim3(256), 0, st, z, D, n, ld, sigma, seed, first);
    return hipGetLastError();
}

hipError_t launch_nsf_backward(const NsfBackArgs& a, int n_cu, hipStream_t st) {
    hipLaunchKernelGGL(dmc_nsf_backward_kernel, dim3(grid_for(a.n, n_cu)), dim3(256), 0, st, a);
    return hipGetLastError();
}

int nsf_outer_chunks(int64_t n) { return (int)((n + OUTER_CHUNK - 1) / OUTER_CHUNK); }

hipError_t launch_nsf_outer(const float* A, int rowsA, const float* B, int rowsB, int64_t n, float* partial,
                            hipStream_t st) {
    if (rowsB > 32 || rowsA < 1 || rowsB < 0) return hipErrorInvalidValue;
    if (n <= 0) return hipSuccess;
    const int tiles = (rowsA + 31) / 32;
    const dim3 grid((tiles + OUTER_TILES - 1) / OUTER_TILES, nsf_outer_chunks(n));
    hipLaunchKernelGGL(dmc_nsf_outer_kernel, grid, dim3(64 * OUTER_WAVES), 0, st, A, rowsA, B, rowsB, n, partial);
    return hipGetLastError();
}

hipError_t launch_nsf_outer_fold(const float* partial, int rowsA, int rowsB, int64_t n, float* grad, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int t = rowsA * (rowsB + 1);
    hipLaunchKernelGGL(dmc_nsf_outer_fold_kernel, dim3((t + 63) / 64), dim3(1024), 0, st, partial, rowsA, rowsB,
                       nsf_outer_chunks(n), grad);
    return hipGetLastError();
}

hipError_t launch_nsf_loss(const float* w, const float* lq, int64_t n, double* out, int, hipStream_t st) {
    hipLaunchKernelGGL(dmc_nsf_loss_kernel, dim3(1), dim3(1024), 0, st, w, lq, n, out);
    return hipGetLastError();
}

hipError_t launch_nsf_adam(float* params, float* m, float* v, const float* grad, int64_t count, int64_t step, float lr,
                           hipStream_t st) {
    const float c1 = 1.0f / (1.0f - powf(0.9f, (float)step));
    const float c2 = 1.0f / (1.0f - powf(0.999f, (float)step));
    const int64_t want = (count + 255) / 256;
    hipLaunchKernelGGL(dmc_nsf_adam_kernel, dim3((unsigned)(want < 2048 ? want : 2048)), dim3(256), 0, st, params, m, v,
                       grad, count, lr, c1, c2);
    return hipGetLastError();
}

}  // namespace dmc
