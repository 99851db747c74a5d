// Argument blocks and launchers of the Markov-chain estimator (independent proposals).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dmc {

struct McmcArgs {
    int64_t n;                // chains
    int S;                    // observable slots per chain ([G][R][K][2], the eval capture layout)
    int R, K;                 // roots and external momenta (root-0 slots define p = |f|)
    int G;
    const float* f_prop;      // [S][ld_prop]: integrand at the proposals
    int64_t ld_prop;
    const float* jac_prop;    // [n]: 1 / q at the proposals
    int64_t offset;           // chain c takes proposal (c + offset) mod n, 0 <= offset < n
    int D;                    // coordinates kept per chain (0: none)
    const float* u_prop;      // [D][ld_u]: the proposals' coordinates (when D > 0)
    int64_t ld_u;
    float* u_state;           // [D][n]
    float* f_state;           // [S][n]
    double* q_state;          // [n]
    double* pi_state;         // [n]
    double alpha;
    uint64_t seed, step;
    int first;                // accept every proposal (initial state)
    // base-space random walk (nullable): the flow's own weights 1 / q_T at the proposals and at the states;
    // chain c's proposal is column c, and the test uses q_T in place of the proposal density
    const float* g_prop;
    const float* g_state;
    unsigned long long* n_acc;
};

struct McmcAccArgs {
    int64_t n;
    int S;
    int n_batches;            // chain batch b: chains [b n / B, (b + 1) n / B)
    const float* f_state;
    const double* q_state;
    const double* pi_state;
    double* partial;          // [blocks per batch][n_batches][S + 1][2]
    int chunk;                // chains per block
};

hipError_t launch_mcmc_accept(const McmcArgs& a, int n_cu, hipStream_t st);

struct McmcTrainArgs {
    int64_t n;
    int S, R, K, G, D;
    const float* f_state;     // [S][n]
    const double* pi_state;   // [n]
    const float* u_state;     // [D][n]
    float* u_out;             // [D][ld_out]
    int64_t ld_out;
    float* w_out;             // [n]
};
hipError_t launch_mcmc_training(const McmcTrainArgs& a, int n_cu, hipStream_t st);
// blocks per chain batch (each block sums `chunk` chains of one batch) for batches of at most n chains
int mcmc_acc_blocks(int64_t n, int* chunk);
hipError_t launch_mcmc_accumulate(const McmcAccArgs& a, int blocks_per_batch, hipStream_t st);

}  // namespace dmc
