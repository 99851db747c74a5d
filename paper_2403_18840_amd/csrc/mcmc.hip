// Markov-chain estimator with independent proposals (Sec. IV, eq. target_distr_nf_mcmc_qft_revised
// and eq. nf_mcmc_estimator_qft_final_revised), one chain per sample lane.
//
// The proposal density q is the sampler's (VEGAS or flow mixture): jac = 1/q at every proposal.
// A sampler may lay its proposals out by index (the defensive mixture puts each component's share
// in one index range), so chain c takes proposal (c + offset) mod n with a fresh uniform offset per
// step: each chain's proposal is then a draw from q itself, whatever the layout.
// The target is pi = alpha q + (1 - alpha) p with p = |f| summed over the root-0 observables
// (every lambda group, external momentum, Re and Im).  A chain's state needs no coordinates (the
// next proposal does not depend on it): only the integrand values f, q and pi at its point.
//   dmc_mcmc_accept_kernel      Metropolis-Hastings test (FP64), state update (values and, when kept,
//                               the proposal's coordinates), accepted count; also the test of a
//                               random-walk move in the flow's base space
//   dmc_mcmc_training_kernel    the states as forward-KL training data: coordinates and w = p / pi
//   dmc_mcmc_accumulate_kernel  per block, sums over its chains of f/pi per slot and of q/pi,
//                               with their squares (FP64, fixed order); the chains fall into
//                               independent batches, each block within one batch, and the partials
//                               fold into per-batch totals like eval partials
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mcmc.hpp"

namespace dmc {

__device__ __forceinline__ void philox_round10(uint32_t c[4], uint32_t k0, uint32_t k1) {
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

// Accept x' with probability min(1, pi(x') q(x) / (pi(x) q(x'))): with u the chain's uniform for this
// step (Philox, key = seed, counter = (chain, step)), x' is taken when u pi(x) q(x') < pi(x') q(x).
__global__ void __launch_bounds__(256) dmc_mcmc_accept_kernel(McmcArgs a) {
    unsigned long long acc = 0;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < a.n; c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t col = c < a.n - a.offset ? c + a.offset : c + a.offset - a.n;
        // p(x') = sum of |f| over the root-0 slots: slot ((g R + 0) K + k) 2 + comp
        double p = 0.0;
        for (int g = 0; g < a.G; ++g)
            for (int s = g * a.R * a.K * 2; s < (g * a.R + 1) * a.K * 2; ++s)
                p += fabs((double)a.f_prop[(int64_t)s * a.ld_prop + col]);
        const double jp = (double)a.jac_prop[col];
        const double qp = 1.0 / jp;
        const double pip = a.alpha * qp + (1.0 - a.alpha) * p;
        // a proposal (or state) whose density or target is not finite and positive is invalid: never
        // taken; a chain without a valid state takes the next valid proposal
        const bool vp = jp > 0.0 && __builtin_isfinite(qp) && __builtin_isfinite(pip) && pip > 0.0;
        const double pis = a.first ? 0.0 : a.pi_state[c], qs = a.first ? 0.0 : a.q_state[c];
        const bool vs = pis > 0.0 && __builtin_isfinite(pis);
        bool take = false;
        if (a.g_prop) {
            // random walk in the flow's base space: in base coordinates the chain's target is pi / q_T and the
            // move is symmetric, so x' is taken when u pi(x) q_T(x') < pi(x') q_T(x); a chain without a valid
            // state (it has no base point) stays
            const double gp = 1.0 / (double)a.g_prop[col], gs = 1.0 / (double)a.g_state[c];
            const bool vg = __builtin_isfinite(gp) && gp > 0.0 && __builtin_isfinite(gs) && gs > 0.0;
            if (vp && vs && vg) {
                uint32_t w[4] = {(uint32_t)c, (uint32_t)((uint64_t)c >> 32), (uint32_t)a.step, (uint32_t)(a.step >> 32)};
                philox_round10(w, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
                const double u = ((double)(w[0] >> 8) + 0.5) * 0x1p-24;
                take = u * pis * gp < pip * gs;
            }
        } else if (vp && !vs) {
            take = true;
        } else if (vp) {
            uint32_t w[4] = {(uint32_t)c, (uint32_t)((uint64_t)c >> 32), (uint32_t)a.step, (uint32_t)(a.step >> 32)};
            philox_round10(w, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
            const double u = ((double)(w[0] >> 8) + 0.5) * 0x1p-24;
            take = u * pis * qp < pip * qs;
        }
        if (a.first && !vp) {
            a.q_state[c] = 0.0;
            a.pi_state[c] = 0.0;  // no valid state yet
        }
        if (take) {
            for (int s = 0; s < a.S; ++s) a.f_state[(int64_t)s * a.n + c] = a.f_prop[(int64_t)s * a.ld_prop + col];
            for (int d = 0; d < a.D; ++d) a.u_state[(int64_t)d * a.n + c] = a.u_prop[(int64_t)d * a.ld_u + col];
            a.q_state[c] = qp;
            a.pi_state[c] = pip;
            ++acc;
        }
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if ((threadIdx.x & 63) == 0 && acc) atomicAdd(a.n_acc, acc);
}

// block (j B + b, s): chains [c0 + j chunk, ...) of batch b = [b n / B, (b + 1) n / B); v = f_s / pi
// (s < S) or q / pi (s = S).  partial[j B + b] is row j, column block b of [blocks][B][S + 1][2]; each block adds
// its step's sums to its own running totals there (steps in order), folded across blocks only when read.
__global__ void __launch_bounds__(256) dmc_mcmc_accumulate_kernel(McmcAccArgs a) {
    const int s = blockIdx.y;
    const int b = (int)(blockIdx.x % (unsigned)a.n_batches), j = (int)(blockIdx.x / (unsigned)a.n_batches);
    const int64_t lo = (int64_t)b * a.n / a.n_batches, hi = (int64_t)(b + 1) * a.n / a.n_batches;
    const int64_t c0 = lo + (int64_t)j * a.chunk;
    const int64_t c1 = c0 + a.chunk < hi ? c0 + a.chunk : hi;
    double s1 = 0.0, s2 = 0.0;
    for (int64_t c = c0 + threadIdx.x; c < c1; c += 256) {
        const double pi = a.pi_state[c];
        const double num = s < a.S ? (double)a.f_state[(int64_t)s * a.n + c] : a.q_state[c];
        const double v = pi > 0.0 ? num / pi : 0.0;  // a chain without a valid state adds nothing
        s1 += v;
        s2 = __builtin_fma(v, v, s2);
    }
    __shared__ double r1[256], r2[256];
    r1[threadIdx.x] = s1;
    r2[threadIdx.x] = s2;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            r1[threadIdx.x] += r1[threadIdx.x + o];
            r2[threadIdx.x] += r2[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t o = ((int64_t)blockIdx.x * (a.S + 1) + s) * 2;
        a.partial[o] += r1[0];
        a.partial[o + 1] += r2[0];
    }
}

// w = p / pi with p = sum of |f| over the root-0 slots of the state (0 without a valid state), and a copy
// of the state's coordinates
__global__ void __launch_bounds__(256) dmc_mcmc_training_kernel(McmcTrainArgs a) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < a.n; c += (int64_t)gridDim.x * blockDim.x) {
        double p = 0.0;
        for (int g = 0; g < a.G; ++g)
            for (int s = g * a.R * a.K * 2; s < (g * a.R + 1) * a.K * 2; ++s)
                p += fabs((double)a.f_state[(int64_t)s * a.n + c]);
        const double pi = a.pi_state[c];
        a.w_out[c] = pi > 0.0 && __builtin_isfinite(pi) ? (float)(p / pi) : 0.0f;
        for (int d = 0; d < a.D; ++d) a.u_out[(int64_t)d * a.ld_out + c] = a.u_state[(int64_t)d * a.n + c];
    }
}

hipError_t launch_mcmc_training(const McmcTrainArgs& a, int n_cu, hipStream_t st) {
    const int64_t want = (a.n + 255) / 256;
    const int64_t cap = (int64_t)n_cu * 8;
    hipLaunchKernelGGL(dmc_mcmc_training_kernel, dim3((unsigned)(want < cap ? want : cap)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_mcmc_accept(const McmcArgs& a, int n_cu, hipStream_t st) {
    const int64_t want = (a.n + 255) / 256;
    const int64_t cap = (int64_t)n_cu * 8;
    hipLaunchKernelGGL(dmc_mcmc_accept_kernel, dim3((unsigned)(want < cap ? want : cap)), dim3(256), 0, st, a);
    return hipGetLastError();
}

int mcmc_acc_blocks(int64_t n, int* chunk) {
    int64_t ch = 4096;
    while ((n + ch - 1) / ch > 1024) ch *= 2;
    *chunk = (int)ch;
    return (int)((n + ch - 1) / ch);
}

hipError_t launch_mcmc_accumulate(const McmcAccArgs& a, int blocks_per_batch, hipStream_t st) {
    hipLaunchKernelGGL(dmc_mcmc_accumulate_kernel, dim3((unsigned)blocks_per_batch * a.n_batches, a.S + 1), dim3(256), 0,
                       st, a);
    return hipGetLastError();
}

}  // namespace dmc
