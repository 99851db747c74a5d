/* Oracle integrand in plain C (test infrastructure): the diagram-by-diagram FP64 evaluation of
 * oracle/integrand.py, for the high orders (5 and 6: 2232 and 31130 diagrams) where the numpy loop
 * over diagrams is too slow for integrals and for per-sample checks of many external momenta.
 *
 * It follows the same definitions, written out again (Sec. II.A eq. sigma_integration; Sec. VI.A
 * eq. ueg_action, eq. interaction_ct; eq. propagator):
 *   W_d(x) = w_d (2 pi)^(-3n) prod_{propagators} G0(|p|^2 - mu, tau_b - tau_a) prod_{interactions} V(|p|^2),
 *   V(q^2) = 8 pi gamma / (q^2 + lambda),
 *   G0(eps, tau) = -exp(-eps tau) (1 - nF(eps)) for 0 < tau < beta, exp(-eps tau) nF(eps) for tau <= 0,
 * evaluated with every exponential bounded (the branches multiplied through by 1 - nF or nF);
 * equal time (both ends on one interaction line) is 0^-.  f(x) = sum_d W_d e^{i w_0 tau_ext(d)},
 * w_0 = pi / beta.  The lines' momenta p = sum_j c_j q_j + c_k k z come from the routed diagram
 * table (the oracle's own routing), passed in as data.  No hoisting, no common subexpressions:
 * each diagram is a plain product of its lines.
 *
 * Derivatives (mode & 1) by forward dual numbers in (mu, lambda, k), the Leibniz rule over the
 * product, as in integrand.diagram_values_dual; with them the magnitudes of each derivative's
 * terms before cancellation (the "absolute" scales there).  For every quantity also
 * sum_d |term_d| C_d, C_d = sum over the diagram's propagators of
 * |eps| (S + beta) + S (|p|^2 + 2 |p| m_p) (integrand.exponent_condition).
 *
 * Output per sample, for q in (value, d/dmu, d/dlambda, d/dk) (derivatives only with mode & 1):
 * Re, Im, sum of magnitudes, sum of magnitudes times C_d.  OpenMP over samples. */
#include <math.h>
#include <stdlib.h>

/* Fermi function without overflow */
static double fermi(double eps, double beta) {
    const double x = beta * eps;
    const double e = exp(-fabs(x));
    return x >= 0 ? e / (1.0 + e) : 1.0 / (1.0 + e);
}

/* free propagator, tau in (-beta, beta), tau == 0 taken as 0^- */
static double g0(double eps, double tau, double beta) {
    if (tau > 0) {
        if (eps >= 0) return -exp(-eps * tau) / (1.0 + exp(-beta * eps));
        return -exp(eps * (beta - tau)) / (1.0 + exp(beta * eps));
    }
    if (eps >= 0) return exp(-eps * (tau + beta)) / (1.0 + exp(-beta * eps));
    return exp(-eps * tau) / (1.0 + exp(beta * eps));
}

/* table: per diagram n_lines rows of (kind, a, b, c_0 .. c_n) with kind 0 = propagator from
 * interaction line a to line b, 1 = interaction; weight[d], ext[d] (the out-vertex's line) */
int oracle_evaluate(int n, int n_diag, int n_lines, const int* table, const double* weight, const int* ext,
                    long long N, const double* x, double k, double beta, double mu, double lam, double gamma,
                    int mode, double* out) {
    const int row = 3 + n + 1;
    const int D = 4 * n - 1;
    const int nq = (mode & 1) ? 4 : 1;
    const double w0 = M_PI / beta;
    const double pref = pow(2.0 * M_PI, -3.0 * n);
    if (n < 1 || n > 6 || n_diag < 1 || N < 0) return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (long long i = 0; i < N; ++i) {
        const double* xi = x + i * D;
        double tau[6];
        tau[0] = 0.0;
        for (int j = 1; j < n; ++j) tau[j] = xi[3 * n + j - 1];
        double qn[6];
        for (int j = 0; j < n; ++j)
            qn[j] = sqrt(xi[3 * j] * xi[3 * j] + xi[3 * j + 1] * xi[3 * j + 1] + xi[3 * j + 2] * xi[3 * j + 2]);
        double acc[16] = {0};
        for (int d = 0; d < n_diag; ++d) {
            const int* L = table + (size_t)d * n_lines * row;
            double v = weight[d] * pref, dmu = 0, dlam = 0, dk = 0;
            double av = fabs(v), amu = 0, alam = 0, ak = 0;
            double cond = 0;
            for (int l = 0; l < n_lines; ++l) {
                const int* r = L + l * row;
                double p[3] = {0, 0, 0}, mp = 0;
                for (int j = 0; j < n; ++j) {
                    const int c = r[3 + j];
                    if (!c) continue;
                    p[0] += c * xi[3 * j];
                    p[1] += c * xi[3 * j + 1];
                    p[2] += c * xi[3 * j + 2];
                    mp += abs(c) * qn[j];
                }
                const int ck = r[3 + n];
                p[2] += ck * k;
                mp += abs(ck) * fabs(k);
                const double p2 = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
                const double dp2dk = 2.0 * ck * p[2];
                double f, fmu = 0, flam = 0, fk, afmu = 0, aflam = 0, afk;
                if (r[0] == 0) {
                    const int a = r[1], b = r[2];
                    const double t = a == b ? 0.0 : tau[b] - tau[a];
                    const double eps = p2 - mu;
                    f = g0(eps, t, beta);
                    const double nf = fermi(eps, beta);
                    /* d G0 / d eps: tau > 0: G0 (beta nF - tau); tau <= 0: G0 (-tau - beta (1 - nF)) */
                    const double dge = t > 0 ? f * (beta * nf - t) : f * (-t - beta * (1.0 - nf));
                    fmu = -dge;
                    fk = dge * dp2dk;
                    const double tp = t > 0 ? t : t + beta;
                    const double lmu = tp + beta * nf;
                    afmu = fabs(f) * lmu;
                    afk = fabs(f) * lmu * fabs(dp2dk);
                    const double S = eps >= 0 ? tp : beta - tp;
                    cond += fabs(eps) * (S + beta) + S * (p2 + 2.0 * sqrt(p2) * mp);
                } else {
                    f = 8.0 * M_PI * gamma / (p2 + lam);
                    flam = -f / (p2 + lam);
                    fk = flam * dp2dk;
                    aflam = fabs(f) / (p2 + lam);
                    afk = aflam * fabs(dp2dk);
                }
                const double af = fabs(f);
                dmu = dmu * f + v * fmu;
                dlam = dlam * f + v * flam;
                dk = dk * f + v * fk;
                amu = amu * af + av * afmu;
                alam = alam * af + av * aflam;
                ak = ak * af + av * afk;
                v *= f;
                av *= af;
            }
            const double ph = w0 * tau[ext[d]];
            const double c = cos(ph), s = sin(ph);
            const double vals[4] = {v, dmu, dlam, dk}, abss[4] = {av, amu, alam, ak};
            for (int q = 0; q < nq; ++q) {
                acc[4 * q] += vals[q] * c;
                acc[4 * q + 1] += vals[q] * s;
                acc[4 * q + 2] += abss[q];
                acc[4 * q + 3] += abss[q] * cond;
            }
        }
        for (int q = 0; q < 4 * nq; ++q) out[i * 4 * nq + q] = acc[q];
    }
    return 0;
}
