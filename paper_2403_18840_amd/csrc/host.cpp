// Host FP64 arithmetic of the estimators (no device): combination of frozen-grid iterations, the
// Markov-chain ratio estimator from the chains' batch sums, and the effective-mass coefficient tables.
#include <cmath>
#include <cstring>
#include <limits>
#include <vector>

#include "../../include/dmc.h"

namespace dmc {
dmc_status set_error(dmc_status s, const char* msg);  // the thread-local error text (api.cpp)
}

extern "C" {

dmc_status dmc_combine_iterations(int32_t n_iter, int32_t n_values, const double* means, const double* errs,
                                  double* mean, double* err, double* chi2_dof) {
    if (!means || !errs || !mean || !err || !chi2_dof) return dmc::set_error(DMC_E_INVALID, "null argument");
    if (n_iter < 1 || n_values < 1) return dmc::set_error(DMC_E_INVALID, "need n_iter >= 1 and n_values >= 1");
    const double nan = std::numeric_limits<double>::quiet_NaN();
    for (int v = 0; v < n_values; ++v) {
        double s = 0.0, e2 = 0.0;
        for (int i = 0; i < n_iter; ++i) {
            s += means[(size_t)i * n_values + v];
            e2 += errs[(size_t)i * n_values + v] * errs[(size_t)i * n_values + v];
        }
        const double m = s / n_iter;
        mean[v] = m;
        err[v] = std::sqrt(e2) / n_iter;
        double c = 0.0;
        bool ok = n_iter >= 2;
        for (int i = 0; i < n_iter && ok; ++i) {
            const double d = means[(size_t)i * n_values + v] - m, e = errs[(size_t)i * n_values + v];
            if (!(e > 0)) ok = false;
            else c += d * d / (e * e);
        }
        chi2_dof[v] = ok ? c / (n_iter - 1) : nan;
    }
    return DMC_OK;
}

dmc_status dmc_chains_ratio(int32_t n_batches, int32_t n_groups, int32_t n_roots, int32_t n_k, const double* sums,
                            int32_t order, const dmc_instance* inst, int32_t n_inst, double* mean, double* err) {
    if (!sums || !inst || !mean || !err) return dmc::set_error(DMC_E_INVALID, "null argument");
    if (n_batches < 2 || n_groups < 1 || n_roots < 1 || n_k < 1 || n_inst < 1 || order < 1)
        return dmc::set_error(DMC_E_INVALID, "need n_batches >= 2 and positive shapes");
    const int S = n_groups * n_roots * n_k * 2;
    // groups by lambda in order of first appearance, as in dmc_eval_batch; factor (gamma / gamma_group)^order
    std::vector<double> lam, gam;
    std::vector<int> grp(n_inst);
    std::vector<double> fac(n_inst);
    for (int i = 0; i < n_inst; ++i) {
        int g = -1;
        for (size_t j = 0; j < lam.size(); ++j)
            if (lam[j] == inst[i].lambda) g = (int)j;
        if (g < 0) {
            g = (int)lam.size();
            lam.push_back(inst[i].lambda);
            gam.push_back(inst[i].gamma);
        }
        grp[i] = g;
        fac[i] = std::pow(inst[i].gamma / gam[g], order);
    }
    if ((int)lam.size() != n_groups) return dmc::set_error(DMC_E_INVALID, "instances do not match n_groups");
    const size_t row = (size_t)(S + 1) * 2;
    double den = 0.0;
    for (int b = 0; b < n_batches; ++b) den += sums[b * row + (size_t)S * 2];
    if (!(den > 0)) return dmc::set_error(DMC_E_NUMERIC, "no measured chain weight");
    // per slot: overall ratio sum_b num_b / sum_b den_b, and the scatter of the batch ratios num_b / den_b
    std::vector<double> m(S), e(S);
    for (int s = 0; s < S; ++s) {
        double num = 0.0, a = 0.0, a2 = 0.0;
        for (int b = 0; b < n_batches; ++b) {
            const double nb = sums[b * row + (size_t)s * 2], db = sums[b * row + (size_t)S * 2];
            num += nb;
            const double rb = db > 0 ? nb / db : 0.0;
            a += rb;
            a2 += rb * rb;
        }
        m[s] = num / den;
        const double mb = a / n_batches;
        const double var = (a2 - n_batches * mb * mb) / (n_batches - 1);
        e[s] = std::sqrt(var > 0 ? var : 0.0) / std::sqrt((double)n_batches);
    }
    // slots [g][r][k][c] -> mean[i][r][k][c]
    for (int i = 0; i < n_inst; ++i)
        for (int r = 0; r < n_roots; ++r)
            for (int k = 0; k < n_k; ++k)
                for (int c = 0; c < 2; ++c) {
                    const int s = ((grp[i] * n_roots + r) * n_k + k) * 2 + c;
                    const size_t o = (((size_t)i * n_roots + r) * n_k + k) * 2 + c;
                    mean[o] = m[s] * fac[i];
                    err[o] = e[s] * std::fabs(fac[i]);
                }
    return DMC_OK;
}

dmc_status dmc_mass_table(int32_t order, const int32_t* root_orders, int32_t n_roots, const double* est, double beta,
                          int32_t* nml, double* sigma, double* a, double* b, int32_t* n_out) {
    if (!root_orders || !est || !nml || !sigma || !a || !b || !n_out) return dmc::set_error(DMC_E_INVALID, "null argument");
    if (order < 1 || n_roots < 1 || !(beta > 0)) return dmc::set_error(DMC_E_INVALID, "need order >= 1, n_roots >= 1, beta > 0");
    const double w0 = M_PI / beta;
    int n = 0;
    for (int r = 0; r < n_roots; ++r) {
        const int m = root_orders[3 * r], l = root_orders[3 * r + 1], e = root_orders[3 * r + 2];
        if (e != 0) continue;
        nml[3 * n] = order;
        nml[3 * n + 1] = m;
        nml[3 * n + 2] = l;
        sigma[n] = est[2 * r];          // Re Sigma^(n,m,l)(k_F, i w_0)
        b[n] = est[2 * r + 1] / w0;     // Im / w_0
        a[n] = 0.0;
        for (int q = 0; q < n_roots; ++q)
            if (root_orders[3 * q] == m && root_orders[3 * q + 1] == l && root_orders[3 * q + 2] == 1)
                a[n] = 0.5 * est[2 * q];  // (m_e / k_F) d Re Sigma / dk, m_e / k_F = 1/2 (eps_k = k^2)
        ++n;
    }
    *n_out = n;
    return DMC_OK;
}

}  // extern "C"

extern "C" {

dmc_status dmc_proposal_select(int32_t n_values, const double* err_flow, const double* err_grid, double t_flow,
                               double t_grid, int64_t nonfinite_flow, double min_gain, int32_t* use_flow,
                               double* gain) {
    if (!err_flow || !err_grid || !use_flow || !gain) return dmc::set_error(DMC_E_INVALID, "null argument");
    if (n_values < 1) return dmc::set_error(DMC_E_INVALID, "need n_values >= 1");
    if (!(t_flow > 0) || !(t_grid > 0) || !std::isfinite(t_flow) || !std::isfinite(t_grid))
        return dmc::set_error(DMC_E_INVALID, "probe times must be positive and finite");
    if (!(min_gain >= 0)) return dmc::set_error(DMC_E_INVALID, "min_gain must be >= 0");
    double vf = 0.0, vg = 0.0;
    for (int v = 0; v < n_values; ++v) {
        vf += err_flow[v] * err_flow[v];
        vg += err_grid[v] * err_grid[v];
    }
    // efficiency of the flow over the grid: (variance x time) of the grid over that of the flow
    double g = 0.0;
    if (std::isfinite(vf) && std::isfinite(vg)) {
        if (vf > 0) g = (vg * t_grid) / (vf * t_flow);
        else g = vg > 0 ? std::numeric_limits<double>::infinity() : 1.0;
    }
    *gain = g;
    *use_flow = (nonfinite_flow == 0 && g >= min_gain) ? 1 : 0;
    return DMC_OK;
}

}  // extern "C"
