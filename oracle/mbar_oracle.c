/*
 * mbar_oracle.c -- plain FP64 CPU oracle of the multistate reweighting used by the
 * REGC method (arXiv:1908.11118, Sec. II.B) to turn the sampled (E, N) of all
 * states into partition-function estimates and averages at any (T, mu).
 *
 * TEST INFRASTRUCTURE ONLY (see regc_oracle.c).  Shares nothing with the HIP path.
 *
 * Reduced potential of a sample n in state s (Sec. II.B, Eq. (8) with the sign of
 * mu*N as the paper fixes it, plus the 3N ln Lambda(T) term of Eq. (1) so that
 * states of different T are consistent with the swap rule):
 *     u_s(n) = beta_s E_n - N_n lnz_s,   lnz_s = beta_s mu_s - 3 ln Lambda(T_s).
 * Self-consistent equations (Sec. II.B, Eq. (9), read in the standard form with
 * the target state in the numerator and all sampled states in the denominator),
 * in log form with f_s = -ln c_s:
 *     log D_n = logsumexp_k [ ln Omega_k + f_k - u_k(n) ]      (k sampled)
 *     f_s     = -logsumexp_n [ -u_s(n) - log D_n ]
 * iterated from f = 0 with the gauge f_{first sampled state} = 0, until the
 * largest change is below tol.  This is the plain S x N_s double loop.
 * Averages at any state t follow Eq. (10)/(11): weights
 *     w_n(t) = exp(f_t - u_t(n) - log D_n),
 * <N>_t = sum w N, p_t(N*) = sum over samples with N = N* of w (Eq. (10) with the
 * indicator of phase N*), phase = the N* of largest p (smallest N* on ties).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

static double lse_pair(double m, double s) { return m + log(s); }

/* logD for every sample */
static void mbar_logd(int S, const double *beta, const double *lnz, const int64_t *omega,
                      const double *f, int64_t ns, const double *e, const int32_t *nn,
                      double *logd, int n_threads)
{
#pragma omp parallel for schedule(static) num_threads(n_threads)
    for (int64_t n = 0; n < ns; ++n) {
        double mx = -INFINITY;
        for (int k = 0; k < S; ++k) {
            if (omega[k] <= 0) continue;
            double v = log((double)omega[k]) + f[k] - (beta[k] * e[n] - (double)nn[n] * lnz[k]);
            if (v > mx) mx = v;
        }
        double sum = 0.0;
        for (int k = 0; k < S; ++k) {
            if (omega[k] <= 0) continue;
            double v = log((double)omega[k]) + f[k] - (beta[k] * e[n] - (double)nn[n] * lnz[k]);
            sum += exp(v - mx);
        }
        logd[n] = lse_pair(mx, sum);
    }
}

/* f_t = -logsumexp_n(-u_t(n) - logD_n) for one state (beta_t, lnz_t) */
static double mbar_free_energy(double beta_t, double lnz_t, int64_t ns, const double *e,
                               const int32_t *nn, const double *logd)
{
    double mx = -INFINITY;
    for (int64_t n = 0; n < ns; ++n) {
        double v = -(beta_t * e[n] - (double)nn[n] * lnz_t) - logd[n];
        if (v > mx) mx = v;
    }
    double sum = 0.0;
    for (int64_t n = 0; n < ns; ++n) {
        double v = -(beta_t * e[n] - (double)nn[n] * lnz_t) - logd[n];
        sum += exp(v - mx);
    }
    return -lse_pair(mx, sum);
}

/* Solves the self-consistent equations.  f (length S) holds the starting point on
 * entry and the solution on exit; logd (length ns) the final log D_n.
 * Returns 0 when converged, -7 otherwise (f then holds the last iterate). */
int orc_mbar_solve(int S, const double *beta, const double *lnz, const int64_t *omega,
                   int64_t ns, const double *e, const int32_t *nn, double tol, int max_iter,
                   double *f, double *logd, int *iters_out, double *delta_out, int n_threads)
{
    double *fn = (double *)malloc(sizeof(double) * S);
    int g = -1;
    for (int k = 0; k < S; ++k)
        if (omega[k] > 0) { g = k; break; }
    int rc = -7, it = 0;
    double delta = INFINITY;
    if (g < 0) { free(fn); return -1; }
    for (it = 0; it < max_iter; ++it) {
        mbar_logd(S, beta, lnz, omega, f, ns, e, nn, logd, n_threads);
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads)
        for (int s = 0; s < S; ++s) fn[s] = mbar_free_energy(beta[s], lnz[s], ns, e, nn, logd);
        double f0 = fn[g];
        delta = 0.0;
        for (int s = 0; s < S; ++s) {
            fn[s] -= f0;
            if (omega[s] > 0) {
                double d = fabs(fn[s] - f[s]);
                if (d > delta) delta = d;
            }
            f[s] = fn[s];
        }
        if (delta < tol) { rc = 0; ++it; break; }
    }
    /* logD consistent with the returned f */
    mbar_logd(S, beta, lnz, omega, f, ns, e, nn, logd, n_threads);
    if (iters_out) *iters_out = it;
    if (delta_out) *delta_out = delta;
    free(fn);
    return rc;
}

/* One sweep of the self-consistent map (no gauge), for the fixed-point tests and
 * the timing of one iteration: f_out[s] = -logsumexp_n(-u_s(n) - logD_n(f_in)). */
void orc_mbar_iterate(int S, const double *beta, const double *lnz, const int64_t *omega,
                      int64_t ns, const double *e, const int32_t *nn, const double *f_in,
                      double *f_out, double *logd, int n_threads)
{
    mbar_logd(S, beta, lnz, omega, f_in, ns, e, nn, logd, n_threads);
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads)
    for (int s = 0; s < S; ++s) f_out[s] = mbar_free_energy(beta[s], lnz[s], ns, e, nn, logd);
}

/* Averages at T target states, given logD of the solved system.
 * p_n: [T][n_max+1] (may be NULL), others [T]. */
void orc_mbar_targets(int T, const double *tbeta, const double *tlnz, int64_t ns, const double *e,
                      const int32_t *nn, const double *logd, int n_max, double *f_t,
                      double *mean_n, double *mean_e, double *mean_e2, double *p_n,
                      int32_t *phase, int n_threads)
{
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads)
    for (int t = 0; t < T; ++t) {
        double ft = mbar_free_energy(tbeta[t], tlnz[t], ns, e, nn, logd);
        double *hist = (double *)calloc((size_t)n_max + 1, sizeof(double));
        double sn = 0.0, se = 0.0, se2 = 0.0;
        for (int64_t n = 0; n < ns; ++n) {
            double w = exp(ft - (tbeta[t] * e[n] - (double)nn[n] * tlnz[t]) - logd[n]);
            sn += w * (double)nn[n];
            se += w * e[n];
            se2 += w * e[n] * e[n];
            if (nn[n] >= 0 && nn[n] <= n_max) hist[nn[n]] += w;
        }
        int best = 0;
        for (int k = 1; k <= n_max; ++k)
            if (hist[k] > hist[best]) best = k;
        f_t[t] = ft;
        mean_n[t] = sn;
        mean_e[t] = se;
        mean_e2[t] = se2;
        phase[t] = best;
        if (p_n)
            for (int k = 0; k <= n_max; ++k) p_n[(int64_t)t * (n_max + 1) + k] = hist[k];
        free(hist);
    }
}

/* Reweighted observables (Sec. II.B, Eq. (11), read with Omega_{l,m} -- all samples
 * of a sampled state -- in the denominator, i.e. the MBAR weights above): for each
 * target t the weights w_n(t); obs [ns][n_obs] per-sample values (any real
 * observable, e.g. histogram counts).
 *   mean [T][n_obs]          = sum_n w_n obs_n                      (<A>_t)
 *   cond [T][n_max+1][n_obs] = sum_{N_n = N} w_n obs_n / p_t(N)    (<A | N>_t;
 *                              0 where p_t(N) = 0)
 * The joint <A chi_N>_t of Eq. (11) as printed is p_t(N) cond.  Either output may
 * be NULL. */
void orc_mbar_observables(int T, const double *tbeta, const double *tlnz, int64_t ns, const double *e,
                          const int32_t *nn, const double *logd, int n_max, const double *obs, int n_obs,
                          double *mean, double *cond, int n_threads)
{
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads)
    for (int t = 0; t < T; ++t) {
        double ft = mbar_free_energy(tbeta[t], tlnz[t], ns, e, nn, logd);
        double *pn = (double *)calloc((size_t)n_max + 1, sizeof(double));
        double *acc = (double *)calloc(((size_t)n_max + 1) * n_obs, sizeof(double));
        for (int64_t n = 0; n < ns; ++n) {
            double w = exp(ft - (tbeta[t] * e[n] - (double)nn[n] * tlnz[t]) - logd[n]);
            pn[nn[n]] += w;
            for (int k = 0; k < n_obs; ++k) acc[(size_t)nn[n] * n_obs + k] += w * obs[(size_t)n * n_obs + k];
        }
        for (int k = 0; k < n_obs; ++k) {
            double m = 0.0;
            for (int N = 0; N <= n_max; ++N) m += acc[(size_t)N * n_obs + k];
            if (mean) mean[(size_t)t * n_obs + k] = m;
        }
        if (cond)
            for (int N = 0; N <= n_max; ++N)
                for (int k = 0; k < n_obs; ++k)
                    cond[((size_t)t * (n_max + 1) + N) * n_obs + k] =
                        pn[N] > 0.0 ? acc[(size_t)N * n_obs + k] / pn[N] : 0.0;
        free(pn);
        free(acc);
    }
}

