// Renormalisation post-processing of the self-energy's Taylor coefficients (host, FP64).
//
// Sec. III.B: the self-energy as a double series in the order-counting parameter xi and the
// chemical-potential shift dmu = sum_i xi^i delta_mu^(i) (eq. sigma_xi_dmu), the counterterms fixed
// order by order at the Fermi surface (eq. counterterm).  Sec. VI.A: the third variable dlambda =
// -xi lambda_R of the Yukawa re-expansion (eq. interaction_ct, eq. sigma_xi_dmu_dlambda), the series
// a(xi) and b(xi) of eq. dsigma_depsilon_series, and m*/m = Z^-1 (1 + a)^-1 with Z^-1 = 1 - b
// (eq. eff_mass_ratio) expanded in xi.
//
// A coefficient table X^(n,m,l) (n >= 1) becomes the series
//     X(xi) = sum xi^(n+l) dmu(xi)^m / m! (-lambda_R)^l / l! X^(n,m,l)   truncated at xi^N.
// Counterterms: the pole of the full propagator stays at the Fermi surface, so delta_mu^(j) is the
// xi^j coefficient of Sigma(k_F); that coefficient involves delta_mu^(i) for i < j only.
#include <cmath>
#include <vector>

#include "../../include/dmc.h"

namespace dmc {
dmc_status set_error(dmc_status s, const char* msg);
}

namespace {

using Poly = std::vector<double>;  // coefficients of xi^0 .. xi^N

Poly mul(const Poly& a, const Poly& b, int N) {
    Poly out(N + 1, 0.0);
    for (int i = 0; i <= N; ++i)
        for (int j = 0; i + j <= N; ++j) out[i + j] += a[i] * b[j];
    return out;
}

double factorial(int k) {
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= i;
    return f;
}

struct Table {
    int n_coef;
    const int32_t* nml;
    const double* v;
};

Poly xi_series(const Table& t, int N, const Poly& dmu, double lam_R) {
    int mmax = 0;
    for (int c = 0; c < t.n_coef; ++c) mmax = std::max(mmax, (int)t.nml[3 * c + 1]);
    std::vector<Poly> pw(mmax + 1);
    pw[0].assign(N + 1, 0.0);
    pw[0][0] = 1.0;
    for (int m = 1; m <= mmax; ++m) pw[m] = mul(pw[m - 1], dmu, N);
    Poly out(N + 1, 0.0);
    for (int c = 0; c < t.n_coef; ++c) {
        const int n = t.nml[3 * c], m = t.nml[3 * c + 1], l = t.nml[3 * c + 2];
        const int s = n + l;
        if (s > N) continue;
        const double w = t.v[c] / factorial(m) * std::pow(-lam_R, l) / factorial(l);
        for (int j = 0; j + s <= N; ++j) out[j + s] += w * pw[m][j];
    }
    return out;
}

}  // namespace

extern "C" dmc_status dmc_effective_mass(int32_t N, double lambda_R, int32_t n_coef, const int32_t* nml,
                                         const double* sigma_fs, const double* a, const double* b, double* delta_mu,
                                         double* a_xi, double* b_xi, double* mass, double* mass_partial) {
    if (N < 1 || N > 32) return dmc::set_error(DMC_E_INVALID, "N must be in 1..32");
    if (n_coef < 0 || (n_coef > 0 && (!nml || !sigma_fs || !a || !b)) || !delta_mu || !a_xi || !b_xi || !mass ||
        !mass_partial)
        return dmc::set_error(DMC_E_INVALID, "null argument");
    if (!(lambda_R >= 0.0)) return dmc::set_error(DMC_E_INVALID, "lambda_R must be >= 0");
    for (int c = 0; c < n_coef; ++c)
        if (nml[3 * c] < 1 || nml[3 * c + 1] < 0 || nml[3 * c + 2] < 0)
            return dmc::set_error(DMC_E_INVALID, "coefficients need n >= 1, m >= 0, l >= 0");
    Poly d(N + 1, 0.0);
    for (int j = 1; j <= N; ++j) {
        Poly known(d.begin(), d.begin() + j);
        known.resize(j + 1, 0.0);
        d[j] = xi_series(Table{n_coef, nml, sigma_fs}, j, known, lambda_R)[j];
    }
    const Poly A = xi_series(Table{n_coef, nml, a}, N, d, lambda_R);
    const Poly B = xi_series(Table{n_coef, nml, b}, N, d, lambda_R);
    // 1 / (1 + A(xi)) with A(0) = 0: sum_j (-A)^j
    Poly inv(N + 1, 0.0), p(N + 1, 0.0), negA(N + 1, 0.0);
    inv[0] = p[0] = 1.0;
    for (int j = 0; j <= N; ++j) negA[j] = -A[j];
    for (int j = 0; j < N; ++j) {
        p = mul(p, negA, N);
        for (int i = 0; i <= N; ++i) inv[i] += p[i];
    }
    Poly oneB(N + 1, 0.0);
    for (int j = 0; j <= N; ++j) oneB[j] = -B[j];
    oneB[0] += 1.0;
    const Poly M = mul(oneB, inv, N);
    double acc = 0.0;
    for (int j = 0; j <= N; ++j) {
        delta_mu[j] = d[j];
        a_xi[j] = A[j];
        b_xi[j] = B[j];
        mass[j] = M[j];
        acc += M[j];
        mass_partial[j] = acc;
    }
    return DMC_OK;
}
