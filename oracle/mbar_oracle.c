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

/* f_t = -logsumexp_n(ln c_n - u_t(n) - logD_n) for one state (beta_t, lnz_t); c_n is
 * the multiplicity of sample n (cnt == NULL: every sample once; c_n = 0 drops it) */
static double mbar_free_energy(double beta_t, double lnz_t, int64_t ns, const double *e,
                               const int32_t *nn, const double *logd, const int32_t *cnt)
{
    double mx = -INFINITY;
    for (int64_t n = 0; n < ns; ++n) {
        if (cnt && cnt[n] == 0) continue;
        double v = -(beta_t * e[n] - (double)nn[n] * lnz_t) - logd[n] + (cnt ? log((double)cnt[n]) : 0.0);
        if (v > mx) mx = v;
    }
    double sum = 0.0;
    for (int64_t n = 0; n < ns; ++n) {
        if (cnt && cnt[n] == 0) continue;
        double v = -(beta_t * e[n] - (double)nn[n] * lnz_t) - logd[n] + (cnt ? log((double)cnt[n]) : 0.0);
        sum += exp(v - mx);
    }
    return -lse_pair(mx, sum);
}

/* Solves the self-consistent equations with sample multiplicities cnt (NULL: each
 * sample once); omega[k] must be the multiplicity-weighted sample count of state k.
 * f (length S) holds the starting point on entry and the solution on exit; logd
 * (length ns) the final log D_n.  Returns 0 when converged, -7 otherwise (f then
 * holds the last iterate). */
static int mbar_solve_w(int S, const double *beta, const double *lnz, const int64_t *omega,
                        int64_t ns, const double *e, const int32_t *nn, const int32_t *cnt, double tol,
                        int max_iter, double *f, double *logd, int *iters_out, double *delta_out, int n_threads)
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
        for (int s = 0; s < S; ++s) fn[s] = mbar_free_energy(beta[s], lnz[s], ns, e, nn, logd, cnt);
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

int orc_mbar_solve(int S, const double *beta, const double *lnz, const int64_t *omega,
                   int64_t ns, const double *e, const int32_t *nn, double tol, int max_iter,
                   double *f, double *logd, int *iters_out, double *delta_out, int n_threads)
{
    return mbar_solve_w(S, beta, lnz, omega, ns, e, nn, NULL, tol, max_iter, f, logd, iters_out, delta_out,
                        n_threads);
}

/* One sweep of the self-consistent map (no gauge), for the fixed-point tests and
 * the timing of one iteration: f_out[s] = -logsumexp_n(-u_s(n) - logD_n(f_in)). */
void orc_mbar_iterate(int S, const double *beta, const double *lnz, const int64_t *omega,
                      int64_t ns, const double *e, const int32_t *nn, const double *f_in,
                      double *f_out, double *logd, int n_threads)
{
    mbar_logd(S, beta, lnz, omega, f_in, ns, e, nn, logd, n_threads);
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads)
    for (int s = 0; s < S; ++s) f_out[s] = mbar_free_energy(beta[s], lnz[s], ns, e, nn, logd, NULL);
}

/* Averages at T target states, given logD of the solved system; sample n counts
 * cnt[n] times (cnt == NULL: once).  p_n: [T][n_max+1] (may be NULL), others [T]. */
static void mbar_targets_w(int T, const double *tbeta, const double *tlnz, int64_t ns, const double *e,
                           const int32_t *nn, const int32_t *cnt, const double *logd, int n_max, double *f_t,
                           double *mean_n, double *mean_e, double *mean_e2, double *p_n,
                           int32_t *phase, int n_threads)
{
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads)
    for (int t = 0; t < T; ++t) {
        double ft = mbar_free_energy(tbeta[t], tlnz[t], ns, e, nn, logd, cnt);
        double *hist = (double *)calloc((size_t)n_max + 1, sizeof(double));
        double sn = 0.0, se = 0.0, se2 = 0.0;
        for (int64_t n = 0; n < ns; ++n) {
            if (cnt && cnt[n] == 0) continue;
            double w = (cnt ? (double)cnt[n] : 1.0) * exp(ft - (tbeta[t] * e[n] - (double)nn[n] * tlnz[t]) - logd[n]);
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

void orc_mbar_targets(int T, const double *tbeta, const double *tlnz, int64_t ns, const double *e,
                      const int32_t *nn, const double *logd, int n_max, double *f_t,
                      double *mean_n, double *mean_e, double *mean_e2, double *p_n,
                      int32_t *phase, int n_threads)
{
    mbar_targets_w(T, tbeta, tlnz, ns, e, nn, NULL, logd, n_max, f_t, mean_n, mean_e, mean_e2, p_n, phase,
                   n_threads);
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
        double ft = mbar_free_energy(tbeta[t], tlnz[t], ns, e, nn, logd, NULL);
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


/* ------------------------------------------------------------------------- */
/* Errors of the estimates.  The paper gives none; the definitions below are  */
/* the readings this project takes, applied identically by the HIP library.  */
/* ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]);

/* Direct estimate at every sampled state s: the mean of N over the samples held by
 * s, and its standard error by batch means -- the series of s (its samples in the
 * order given) cut into n_batches batches, batch b holding series positions
 * floor(b n_s / B) .. floor((b+1) n_s / B) - 1; SE = sqrt(var(batch means) / B) with
 * the (B - 1) variance.  mean and se are NaN for a state with fewer than B samples. */
void orc_batch_means(int S, int64_t ns, const int32_t *st, const int32_t *nn, int n_batches, double *mean,
                     double *se)
{
    int64_t *count = (int64_t *)calloc((size_t)S, sizeof(int64_t));
    int64_t *rank = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ns > 0 ? ns : 1));
    double *bsum = (double *)calloc((size_t)S * n_batches, sizeof(double));
    int64_t *bcnt = (int64_t *)calloc((size_t)S * n_batches, sizeof(int64_t));
    double *total = (double *)calloc((size_t)S, sizeof(double));
    for (int64_t i = 0; i < ns; ++i) rank[i] = count[st[i]]++;
    for (int64_t i = 0; i < ns; ++i) {
        const int s = st[i];
        /* batch b holds series positions floor(b n / B) .. floor((b + 1) n / B) - 1 */
        int b = 0;
        while ((int64_t)(b + 1) * count[s] / n_batches <= rank[i]) ++b;
        bsum[(size_t)s * n_batches + b] += (double)nn[i];
        bcnt[(size_t)s * n_batches + b] += 1;
        total[s] += (double)nn[i];
    }
    for (int s = 0; s < S; ++s) {
        if (count[s] < n_batches) {
            mean[s] = NAN;
            se[s] = NAN;
            continue;
        }
        mean[s] = total[s] / (double)count[s];
        double mb = 0.0;
        for (int b = 0; b < n_batches; ++b) mb += bsum[(size_t)s * n_batches + b] / (double)bcnt[(size_t)s * n_batches + b];
        mb /= n_batches;
        double v = 0.0;
        for (int b = 0; b < n_batches; ++b) {
            const double d = bsum[(size_t)s * n_batches + b] / (double)bcnt[(size_t)s * n_batches + b] - mb;
            v += d * d;
        }
        se[s] = sqrt(v / (double)(n_batches - 1) / (double)n_batches);
    }
    free(count);
    free(rank);
    free(bsum);
    free(bcnt);
    free(total);
}

/* Moving-block bootstrap over records (a record = record_size consecutive samples,
 * e.g. one sample of every walker of a run).  Replicate b of R records with blocks of
 * `block` records: ceil(R / block) blocks, block j starting at record
 * floor(w (R - block + 1) / 2^32), w = word 0 of Philox block (j, b, 0xFFFFFFFE, 7)
 * keyed by seed; the blocks are concatenated and cut to R records.  mult[r] = how
 * often record r occurs in the replicate. */
void orc_boot_multiplicity(int64_t R, int64_t block, int b, uint64_t seed, int32_t *mult)
{
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    const int64_t nb = (R + block - 1) / block;
    for (int64_t r = 0; r < R; ++r) mult[r] = 0;
    for (int64_t j = 0; j < nb; ++j) {
        const uint32_t ctr[4] = {(uint32_t)j, (uint32_t)b, 0xFFFFFFFEu, 7u};
        uint32_t out[4];
        orc_philox4x32_10(ctr, key, out);
        const int64_t start = (int64_t)(((uint64_t)out[0] * (uint64_t)(R - block + 1)) >> 32);
        for (int64_t k = 0; k < block && j * block + k < R; ++k) mult[start + k] += 1;
    }
}

/* Standard errors at T target states from n_boot bootstrap replicates: each
 * replicate re-solves the self-consistent equations with the samples weighted by
 * their record's multiplicity (started from f_start, the solution of the full data)
 * and re-evaluates <N>, <E>, <E^2> and C = beta^2 (<E^2> - <E>^2) at the targets.
 * se_n, se_c [T] = standard deviations over the replicates ((n_boot - 1) in the
 * denominator).  rep_n, rep_c [n_boot][T] (may be NULL) receive the replicate values.
 * Returns 0, or -7 if a replicate's solve did not converge (the SEs still come from
 * the last iterates). */
int orc_mbar_bootstrap(int S, const double *beta, const double *lnz, int64_t ns, const double *e, const int32_t *nn,
                       const int32_t *st, int64_t record_size, int64_t block, int n_boot, uint64_t seed,
                       const double *f_start, double tol, int max_iter, int T, const double *tbeta,
                       const double *tlnz, int n_max, double *se_n, double *se_c, double *rep_n, double *rep_c,
                       int n_threads)
{
    const int64_t R = ns / record_size;
    int32_t *mult = (int32_t *)malloc(sizeof(int32_t) * (size_t)R);
    int32_t *cnt = (int32_t *)malloc(sizeof(int32_t) * (size_t)ns);
    int64_t *omega = (int64_t *)malloc(sizeof(int64_t) * (size_t)S);
    double *f = (double *)malloc(sizeof(double) * (size_t)S);
    double *logd = (double *)malloc(sizeof(double) * (size_t)ns);
    double *ft = (double *)malloc(sizeof(double) * (size_t)T), *mn = (double *)malloc(sizeof(double) * (size_t)T);
    double *me = (double *)malloc(sizeof(double) * (size_t)T), *me2 = (double *)malloc(sizeof(double) * (size_t)T);
    int32_t *ph = (int32_t *)malloc(sizeof(int32_t) * (size_t)T);
    double *vn = (double *)malloc(sizeof(double) * (size_t)n_boot * T);
    double *vc = (double *)malloc(sizeof(double) * (size_t)n_boot * T);
    int rc = 0;
    for (int b = 0; b < n_boot; ++b) {
        orc_boot_multiplicity(R, block, b, seed, mult);
        for (int k = 0; k < S; ++k) omega[k] = 0;
        for (int64_t i = 0; i < ns; ++i) {
            cnt[i] = mult[i / record_size];
            omega[st[i]] += cnt[i];
        }
        for (int k = 0; k < S; ++k) f[k] = f_start[k];
        if (mbar_solve_w(S, beta, lnz, omega, ns, e, nn, cnt, tol, max_iter, f, logd, NULL, NULL, n_threads) != 0)
            rc = -7;
        mbar_targets_w(T, tbeta, tlnz, ns, e, nn, cnt, logd, n_max, ft, mn, me, me2, NULL, ph, n_threads);
        for (int t = 0; t < T; ++t) {
            vn[(size_t)b * T + t] = mn[t];
            vc[(size_t)b * T + t] = tbeta[t] * tbeta[t] * (me2[t] - me[t] * me[t]);
        }
    }
    for (int t = 0; t < T; ++t) {
        double an = 0.0, ac = 0.0;
        for (int b = 0; b < n_boot; ++b) {
            an += vn[(size_t)b * T + t];
            ac += vc[(size_t)b * T + t];
        }
        an /= n_boot;
        ac /= n_boot;
        double qn = 0.0, qc = 0.0;
        for (int b = 0; b < n_boot; ++b) {
            const double dn = vn[(size_t)b * T + t] - an, dc = vc[(size_t)b * T + t] - ac;
            qn += dn * dn;
            qc += dc * dc;
        }
        se_n[t] = sqrt(qn / (double)(n_boot - 1));
        se_c[t] = sqrt(qc / (double)(n_boot - 1));
    }
    if (rep_n)
        for (size_t q = 0; q < (size_t)n_boot * T; ++q) rep_n[q] = vn[q];
    if (rep_c)
        for (size_t q = 0; q < (size_t)n_boot * T; ++q) rep_c[q] = vc[q];
    free(mult);
    free(cnt);
    free(omega);
    free(f);
    free(logd);
    free(ft);
    free(mn);
    free(me);
    free(me2);
    free(ph);
    free(vn);
    free(vc);
    return rc;
}

/* Configurational heat capacity at constant mu (a reading: the paper's maps give
 * none), C_t = beta_t^2 (<E^2>_t - <E>_t^2), and coverage theta_t = <N>_t / n_sites
 * in monolayers of the n_sites surface sites. */
void orc_heat_capacity_coverage(int T, const double *tbeta, const double *mean_n, const double *mean_e,
                                const double *mean_e2, double n_sites, double *heat_cap, double *coverage)
{
    for (int t = 0; t < T; ++t) {
        heat_cap[t] = tbeta[t] * tbeta[t] * (mean_e2[t] - mean_e[t] * mean_e[t]);
        coverage[t] = mean_n[t] / n_sites;
    }
}
