// mbar.hip -- multistate reweighting of REGC samples (arXiv:1908.11118, Sec. II.B).
//
// Reduced potential of sample n in state s = (l, m):  u_s(n) = beta_l E_n - N_n ln z_lm
// (Eq. (8) with the paper's sign of mu N plus the 3N ln Lambda(T) term of Eq. (1)).
// Self-consistent equations (Eq. (9)) in log form, f_s = -ln c_s:
//     log D_n = logsumexp_k [ln Omega_k + f_k - u_k(n)],   f_s = -logsumexp_n [-u_s(n) - log D_n].
//
// On a T x mu product grid the state sum factorises exactly (the algebra is
// ours, not the paper's):
//     D_n = sum_l exp(-beta_l E_n) A_l(N_n),       A_l(N) = sum_m Omega_lm exp(f_lm + N ln z_lm),
//     exp(-f_lm) = sum_N z_lm^N P_l(N) / A_l(N),   P_l(N) = sum_{n: N_n = N} p_l(n),
// where p_l(n) = exp(-beta_l E_n) A_l(N_n) / D_n is the softmax over temperatures of
// x_l(n) = -beta_l E_n + log A_l(N_n).  One iteration therefore costs L exponentials
// per sample instead of 2 L M, and every partial sum lies in [0, count]: no overflow.
// Samples are sorted by N once (stable radix sort) and cut into chunks of one N
// each; each chunk writes its L partial sums and they are added in chunk order,
// so results are deterministic.
//
// Averages at a target (T', mu'): with y(n) = -beta' E_n - log D_n,
//     G(N) = logsumexp_{n: N_n = N} y(n),   P(N) proportional to exp(N ln z' + G(N)),
//     <N> = sum N P(N),  <E^k> = sum_N P(N) [sum_{N_n=N} E_n^k e^{y}] / [sum_{N_n=N} e^{y}],
//     f' = -logsumexp_N (N ln z' + G(N)),  phase = argmax_N P(N) (Eq. (10)/(11), smallest N on ties).
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <deque>
#include <mutex>
#include <vector>

#include "host_util.h"
#include "philox_dev.h"
#include "regc_dev.h"

namespace regc {

constexpr int kChunk = 2048;
constexpr int kMbarThreads = 256;
constexpr int kMaxL = 64;

__global__ void mbar_count(int64_t ns, const int32_t *n, const int32_t *st, int nN, int S,
                           unsigned long long *omega, unsigned long long *seg, int *bad)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ns; i += (int64_t)gridDim.x * blockDim.x) {
        const int N = n[i], s = st[i];
        if (N < 0 || N >= nN || s < 0 || s >= S) {
            atomicOr(bad, 1);
            continue;
        }
        atomicAdd(omega + s, 1ull);
        atomicAdd(seg + N, 1ull);
    }
}

__global__ void mbar_iota_gather(int64_t ns, const int32_t *n_in, uint32_t *keys, int32_t *idx)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ns; i += (int64_t)gridDim.x * blockDim.x) {
        keys[i] = (uint32_t)n_in[i];
        idx[i] = (int32_t)i;
    }
}

__global__ void mbar_gather_e(int64_t ns, const int32_t *perm, const double *e_in, double *e_out)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ns; i += (int64_t)gridDim.x * blockDim.x)
        e_out[i] = e_in[perm[i]];
}

// log A_l(N) for every l (block) and N (threads)
__global__ void mbar_loga(int M, int nN, const double *lnomega, const double *f, const double *lnz, double *logA)
{
    const int l = blockIdx.x;
    for (int N = threadIdx.x; N < nN; N += blockDim.x) {
        double mx = -INFINITY;
        for (int m = 0; m < M; ++m) {
            const int s = l * M + m;
            if (lnomega[s] == -INFINITY) continue;
            const double v = lnomega[s] + f[s] + (double)N * lnz[s];
            mx = v > mx ? v : mx;
        }
        double sum = 0.0;
        if (mx != -INFINITY)
            for (int m = 0; m < M; ++m) {
                const int s = l * M + m;
                if (lnomega[s] == -INFINITY) continue;
                sum += exp(lnomega[s] + f[s] + (double)N * lnz[s] - mx);
            }
        logA[(size_t)l * nN + N] = mx == -INFINITY ? -INFINITY : mx + log(sum);
    }
}

__device__ __forceinline__ double wsum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// One chunk (samples of a single N) per block: softmax over temperatures per
// sample, partial sums of p_l(n) per chunk; log D_n when requested.
// WEIGHTED: sample i counts wgt[i] times (bootstrap replicates; wgt in sorted order).
template <int LMAX, bool WEIGHTED>
__global__ void __launch_bounds__(kMbarThreads) mbar_chunk(int L, int nN, const double *beta_l, const double *logA,
                                                        const double *e, const int *chunk_n, const int *chunk_b,
                                                        const int *chunk_e, double *partial, double *logd_out,
                                                        const double *wgt)
{
    __shared__ double red[kMbarThreads / 64][LMAX];
    const int c = blockIdx.x;
    const int N = chunk_n[c];
    double la[LMAX], nb[LMAX], acc[LMAX];
#pragma unroll
    for (int l = 0; l < LMAX; ++l) {
        la[l] = l < L ? logA[(size_t)l * nN + N] : -INFINITY;
        nb[l] = l < L ? -beta_l[l] : 0.0;
        acc[l] = 0.0;
    }
    const int end = chunk_e[c];
    for (int i = chunk_b[c] + threadIdx.x; i < end; i += blockDim.x) {
        const double E = e[i];
        double x[LMAX];
        double mx = -INFINITY;
#pragma unroll
        for (int l = 0; l < LMAX; ++l) {
            x[l] = l < L ? nb[l] * E + la[l] : -INFINITY;
            mx = x[l] > mx ? x[l] : mx;
        }
        double sum = 0.0;
#pragma unroll
        for (int l = 0; l < LMAX; ++l) {
            x[l] = l < L ? exp(x[l] - mx) : 0.0;
            sum += x[l];
        }
        const double inv = WEIGHTED ? wgt[i] / sum : 1.0 / sum;
#pragma unroll
        for (int l = 0; l < LMAX; ++l) acc[l] += x[l] * inv;
        if (logd_out) logd_out[i] = mx + log(sum);
    }
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
#pragma unroll
    for (int l = 0; l < LMAX; ++l) {
        const double v = wsum(acc[l]);
        if (lane == 0) red[wave][l] = v;
    }
    __syncthreads();
    for (int l = threadIdx.x; l < L; l += blockDim.x) {
        double v = 0.0;
        for (int wv = 0; wv < kMbarThreads / 64; ++wv) v += red[wv][l];
        partial[(size_t)c * L + l] = v;
    }
}

// New free energies: one block per temperature l.
__global__ void mbar_fnew(int L, int M, int nN, const double *partial, const int *seg_c0, const int *seg_c1,
                          const double *logA, const double *lnz, double *fnew)
{
    extern __shared__ double logB[];
    const int l = blockIdx.x;
    for (int N = threadIdx.x; N < nN; N += blockDim.x) {
        double P = 0.0;
        for (int c = seg_c0[N]; c < seg_c1[N]; ++c) P += partial[(size_t)c * L + l];
        logB[N] = P > 0.0 ? log(P) - logA[(size_t)l * nN + N] : -INFINITY;
    }
    __syncthreads();
    for (int m = threadIdx.x; m < M; m += blockDim.x) {
        const double lz = lnz[l * M + m];
        double mx = -INFINITY;
        for (int N = 0; N < nN; ++N) {
            if (logB[N] == -INFINITY) continue;
            const double v = (double)N * lz + logB[N];
            mx = v > mx ? v : mx;
        }
        double sum = 0.0;
        for (int N = 0; N < nN; ++N) {
            if (logB[N] == -INFINITY) continue;
            sum += exp((double)N * lz + logB[N] - mx);
        }
        fnew[l * M + m] = -(mx + log(sum));
    }
}

// Gauge (f = 0 at state g) and max |delta f| over sampled states; f <- fnew.
__global__ void mbar_gauge(int S, int g, const double *lnomega, double *fnew, double *f, double *delta)
{
    __shared__ double red[16];
    const double f0 = fnew[g];
    double d = 0.0;
    for (int s = threadIdx.x; s < S; s += blockDim.x) {
        const double v = fnew[s] - f0;
        if (lnomega[s] != -INFINITY) {
            const double a = fabs(v - f[s]);
            d = (a > d || a != a) ? a : d;           // a NaN propagates: the host must see it
        }
        f[s] = v;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double t = __shfl_xor(d, o);
        d = (t > d || t != t) ? t : d;
    }
    if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = d;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int k = 0; k < (int)(blockDim.x / 64); ++k) m = (red[k] > m || red[k] != red[k]) ? red[k] : m;
        *delta = m;
    }
}

// Target temperatures: per chunk and target temperature the online (max, s0, s1, s2).
__global__ void __launch_bounds__(kMbarThreads) mbar_target_chunk(int nT, const double *tbeta, const double *e,
                                                               const double *logd, const int *chunk_b,
                                                               const int *chunk_e, double *tpart,
                                                               const double *wgt)
{
    __shared__ double red[kMbarThreads / 64][4];
    const int c = blockIdx.x;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    for (int t = 0; t < nT; ++t) {
        const double b = tbeta[t];
        double mx = -INFINITY, s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int i = chunk_b[c] + threadIdx.x; i < chunk_e[c]; i += blockDim.x) {
            const double E = e[i];
            const double y = -b * E - logd[i];
            if (y > mx) {
                const double sc = exp(mx - y);
                s0 *= sc; s1 *= sc; s2 *= sc;
                mx = y;
            }
            const double w = wgt ? wgt[i] * exp(y - mx) : exp(y - mx);
            s0 += w; s1 += w * E; s2 += w * E * E;
        }
        // wave combine
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double om = __shfl_xor(mx, o), o0 = __shfl_xor(s0, o), o1 = __shfl_xor(s1, o),
                         o2 = __shfl_xor(s2, o);
            const double nm = om > mx ? om : mx;
            const double a = nm == -INFINITY ? 0.0 : exp(mx - nm), bb = nm == -INFINITY ? 0.0 : exp(om - nm);
            s0 = s0 * a + o0 * bb; s1 = s1 * a + o1 * bb; s2 = s2 * a + o2 * bb;
            mx = nm;
        }
        if (lane == 0) { red[wave][0] = mx; red[wave][1] = s0; red[wave][2] = s1; red[wave][3] = s2; }
        __syncthreads();
        if (threadIdx.x == 0) {
            double M = -INFINITY;
            for (int k = 0; k < kMbarThreads / 64; ++k) M = red[k][0] > M ? red[k][0] : M;
            double a0 = 0, a1 = 0, a2 = 0;
            if (M != -INFINITY)
                for (int k = 0; k < kMbarThreads / 64; ++k) {
                    if (red[k][0] == -INFINITY) continue;
                    const double sc = exp(red[k][0] - M);
                    a0 += red[k][1] * sc; a1 += red[k][2] * sc; a2 += red[k][3] * sc;
                }
            double *o = tpart + ((size_t)c * nT + t) * 4;
            o[0] = M; o[1] = a0; o[2] = a1; o[3] = a2;
        }
        __syncthreads();
    }
}

// Per target temperature (block): combine chunk partials by N, then every mu'.
__global__ void mbar_target_eval(int nT, int nMu, int nN, const double *tpart, const int *seg_c0, const int *seg_c1,
                                 const double *tlnz, double *f, double *mean_n, double *mean_e, double *mean_e2,
                                 double *p_n, int32_t *phase)
{
    extern __shared__ double sh[];
    double *G = sh, *E1 = sh + nN, *E2 = sh + 2 * nN;
    const int t = blockIdx.x;
    for (int N = threadIdx.x; N < nN; N += blockDim.x) {
        double M = -INFINITY;
        for (int c = seg_c0[N]; c < seg_c1[N]; ++c) {
            const double m = tpart[((size_t)c * nT + t) * 4];
            M = m > M ? m : M;
        }
        double a0 = 0, a1 = 0, a2 = 0;
        if (M != -INFINITY)
            for (int c = seg_c0[N]; c < seg_c1[N]; ++c) {
                const double *o = tpart + ((size_t)c * nT + t) * 4;
                if (o[0] == -INFINITY) continue;
                const double sc = exp(o[0] - M);
                a0 += o[1] * sc; a1 += o[2] * sc; a2 += o[3] * sc;
            }
        G[N] = (M == -INFINITY || a0 <= 0.0) ? -INFINITY : M + log(a0);
        E1[N] = a0 > 0.0 ? a1 / a0 : 0.0;
        E2[N] = a0 > 0.0 ? a2 / a0 : 0.0;
    }
    __syncthreads();
    for (int m = threadIdx.x; m < nMu; m += blockDim.x) {
        const int k = t * nMu + m;
        const double lz = tlnz[k];
        double mx = -INFINITY;
        int best = 0;
        for (int N = 0; N < nN; ++N) {
            if (G[N] == -INFINITY) continue;
            const double v = (double)N * lz + G[N];
            if (v > mx) { mx = v; best = N; }
        }
        double sum = 0.0;
        for (int N = 0; N < nN; ++N)
            if (G[N] != -INFINITY) sum += exp((double)N * lz + G[N] - mx);
        const double lse = mx + log(sum);
        double sn = 0, se = 0, se2 = 0;
        for (int N = 0; N < nN; ++N) {
            const double p = G[N] == -INFINITY ? 0.0 : exp((double)N * lz + G[N] - lse);
            sn += p * (double)N; se += p * E1[N]; se2 += p * E2[N];
            if (p_n) p_n[(size_t)k * nN + N] = p;
        }
        if (f) f[k] = -lse;
        mean_n[k] = sn;
        if (mean_e) mean_e[k] = se;
        if (mean_e2) mean_e2[k] = se2;
        if (phase) phase[k] = best;
    }
}

// Observables: gather into sorted order
__global__ void mbar_gather_obs(int64_t ns, int n_obs, const int32_t *perm, const uint32_t *in, uint32_t *out)
{
    const int64_t total = ns * n_obs;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = q / n_obs;
        const int k = (int)(q - i * n_obs);
        out[q] = in[(int64_t)perm[i] * n_obs + k];
    }
}

// Per chunk c (one N) and target temperature t (grid y): the scale mx = max of
// y_i = -beta_t E_i - logD_i, s0 = sum exp(y_i - mx) and s_k = sum exp(y_i - mx) obs_ik,
// every sum in sample order (deterministic).  out[(c nT + t)(n_obs + 2) + {0, 1, 2 + k}].
__global__ void __launch_bounds__(kMbarThreads) mbar_obs_chunk(int nT, int n_obs, const double *tbeta, const double *e,
                                                            const double *logd, const int *chunk_b,
                                                            const int *chunk_e, const uint32_t *obs, double *out)
{
    __shared__ double w[kChunk];
    __shared__ double red[kMbarThreads / 64];
    const int c = blockIdx.x, t = blockIdx.y;
    const int b = chunk_b[c], cnt = chunk_e[c] - b;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const double bt = tbeta[t];
    double mx = -INFINITY;
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
        const double y = -bt * e[b + i] - logd[b + i];
        w[i] = y;
        mx = y > mx ? y : mx;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double v = __shfl_xor(mx, o);
        mx = v > mx ? v : mx;
    }
    if (lane == 0) red[wave] = mx;
    __syncthreads();
    mx = red[0];
    for (int k = 1; k < kMbarThreads / 64; ++k) mx = red[k] > mx ? red[k] : mx;
    __syncthreads();
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) w[i] = exp(w[i] - mx);
    __syncthreads();
    double *o = out + ((size_t)c * nT + t) * (n_obs + 2);
    if (threadIdx.x == 0) {
        double s0 = 0.0;
        for (int i = 0; i < cnt; ++i) s0 += w[i];
        o[0] = mx;
        o[1] = s0;
    }
    for (int k = threadIdx.x; k < n_obs; k += blockDim.x) {
        double acc = 0.0;
        for (int i = 0; i < cnt; ++i) acc += w[i] * (double)obs[(size_t)(b + i) * n_obs + k];
        o[2 + k] = acc;
    }
}

// Per target temperature t (block): the chunks of each N combined in order into the
// conditional average cond[t][N][k] and G(N) = ln sum_{N_n = N} exp(-beta_t E - logD);
// then for every target mu: p(N) = exp(N lnz + G(N) - lse) and mean = sum_N p(N) cond.
__global__ void mbar_obs_eval(int nT, int nMu, int nN, int n_obs, const double *part, const int *seg_c0,
                              const int *seg_c1, const double *tlnz, double *cond, double *mean)
{
    extern __shared__ double sh[];    // G [nN] | p(N) of one mu [nN]
    double *G = sh, *P = sh + nN;
    const int t = blockIdx.x;
    const size_t stride = (size_t)n_obs + 2;
    double *ct = cond + (size_t)t * nN * n_obs;
    // the average conditional on N: chunk partials of one N combined in chunk order
    for (int N = 0; N < nN; ++N) {
        double M = -INFINITY;
        for (int c = seg_c0[N]; c < seg_c1[N]; ++c) {
            const double m = part[((size_t)c * nT + t) * stride];
            M = m > M ? m : M;
        }
        double s0 = 0.0;
        if (M != -INFINITY)
            for (int c = seg_c0[N]; c < seg_c1[N]; ++c) {
                const double *o = part + ((size_t)c * nT + t) * stride;
                if (o[0] != -INFINITY) s0 += o[1] * exp(o[0] - M);
            }
        if (threadIdx.x == 0) G[N] = (M == -INFINITY || s0 <= 0.0) ? -INFINITY : M + log(s0);
        for (int k = threadIdx.x; k < n_obs; k += blockDim.x) {
            double a = 0.0;
            if (M != -INFINITY)
                for (int c = seg_c0[N]; c < seg_c1[N]; ++c) {
                    const double *o = part + ((size_t)c * nT + t) * stride;
                    if (o[0] != -INFINITY) a += o[2 + k] * exp(o[0] - M);
                }
            ct[(size_t)N * n_obs + k] = s0 > 0.0 ? a / s0 : 0.0;
        }
    }
    __syncthreads();
    if (!mean) return;
    // mean at every mu: sum over N of p(N) times the conditional average
    for (int m = 0; m < nMu; ++m) {
        const double lz = tlnz[t * nMu + m];
        if (threadIdx.x == 0) {
            double mx = -INFINITY;
            for (int N = 0; N < nN; ++N)
                if (G[N] != -INFINITY) mx = fmax(mx, (double)N * lz + G[N]);
            double sum = 0.0;
            for (int N = 0; N < nN; ++N)
                if (G[N] != -INFINITY) sum += exp((double)N * lz + G[N] - mx);
            const double lse = mx + log(sum);
            for (int N = 0; N < nN; ++N) P[N] = G[N] == -INFINITY ? 0.0 : exp((double)N * lz + G[N] - lse);
        }
        __syncthreads();
        for (int k = threadIdx.x; k < n_obs; k += blockDim.x) {
            double acc = 0.0;
            for (int N = 0; N < nN; ++N)
                if (P[N] != 0.0) acc += P[N] * ct[(size_t)N * n_obs + k];
            mean[((size_t)t * nMu + m) * n_obs + k] = acc;
        }
        __syncthreads();
    }
}

// ---- errors of the estimates ----
// Batch means: per-state series position of every sample (samples sorted stably by
// state), batch b = floor(rank B / n_s), integer sums of N per (state, batch).
// bad when a state is out of range or an N negative
__global__ void bm_check(int64_t ns, const int32_t *st, const int32_t *n, int S, int *bad)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ns; i += (int64_t)gridDim.x * blockDim.x) {
        const int k = st[i];
        if (k < 0 || k >= S || n[i] < 0) atomicOr(bad, 1);
    }
}

// Start and length of every state's run in the keys sorted by state (lower bounds).
__global__ void bm_bounds(int64_t ns, int S, const uint32_t *sorted_state, int64_t *state_start, int64_t *state_count)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    auto lower = [&](uint32_t key) {
        int64_t lo = 0, hi = ns;
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo) / 2;
            if (sorted_state[mid] < key) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    };
    const int64_t a = lower((uint32_t)s), b = lower((uint32_t)s + 1u);
    state_start[s] = a;
    state_count[s] = b - a;
}

// One workgroup per (state, batch): the batch is a contiguous range of the sorted
// order, its sum of N a block reduction of integers (exact in any order).
__global__ void bm_segments(int B, const int32_t *sorted_idx, const int32_t *n_orig, const int64_t *state_start,
                            const int64_t *state_count, unsigned long long *bsum, unsigned long long *bcnt)
{
    __shared__ unsigned long long part[4];
    const int bin = blockIdx.x, s = bin / B, b = bin % B;
    const int64_t cnt = state_count[s];
    const int64_t lo = state_start[s] + (b * cnt) / B, hi = state_start[s] + ((b + 1) * cnt) / B;
    unsigned long long acc = 0;
    for (int64_t p = lo + threadIdx.x; p < hi; p += blockDim.x) acc += (unsigned long long)n_orig[sorted_idx[p]];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (threadIdx.x % 64 == 0) part[threadIdx.x / 64] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        bsum[bin] = part[0] + part[1] + part[2] + part[3];
        bcnt[bin] = (unsigned long long)(hi - lo);
    }
}

// mean and SE of each state from its batch sums (NaN below B samples); batch b's mean
// is bsum / bcnt, SE = sqrt(sum (m_b - mean(m))^2 / ((B - 1) B)), batches in order.
__global__ void bm_finish(int S, int B, const unsigned long long *bsum, const unsigned long long *bcnt,
                          const int64_t *state_count, double *mean, double *se)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    if (state_count[s] < B) {
        mean[s] = NAN;
        se[s] = NAN;
        return;
    }
    double tot = 0.0, mb = 0.0;
    for (int b = 0; b < B; ++b) {
        tot += (double)bsum[(size_t)s * B + b];
        mb += (double)bsum[(size_t)s * B + b] / (double)bcnt[(size_t)s * B + b];
    }
    mb /= B;
    double v = 0.0;
    for (int b = 0; b < B; ++b) {
        const double d = (double)bsum[(size_t)s * B + b] / (double)bcnt[(size_t)s * B + b] - mb;
        v += d * d;
    }
    mean[s] = tot / (double)state_count[s];
    se[s] = sqrt(v / (double)(B - 1) / (double)B);
}

// Moving-block bootstrap, replicate b: block j (of ceil(R / block)) starts at record
// floor(w (R - block + 1) / 2^32), w = word 0 of Philox block (j, b, 0xFFFFFFFE, 7);
// mult[r] counts the occurrences of record r in the concatenation cut to R records.
__global__ void boot_mult(int64_t R, int64_t block, int b, uint32_t k0, uint32_t k1, int32_t *mult)
{
    const int64_t nb = (R + block - 1) / block;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nb; j += (int64_t)gridDim.x * blockDim.x) {
        const uint4 w = philox4x32_10(make_uint4((uint32_t)j, (uint32_t)b, 0xFFFFFFFEu, 7u), k0, k1);
        const int64_t start = (int64_t)(((uint64_t)w.x * (uint64_t)(R - block + 1)) >> 32);
        for (int64_t k = 0; k < block && j * block + k < R; ++k) atomicAdd(mult + start + k, 1);
    }
}

__global__ void fill_i32(int64_t count, int32_t v, int32_t *x)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = v;
}

__global__ void fill_u64(int64_t count, unsigned long long *x)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = 0ull;
}

// Sample weights of a replicate in sorted order and the weighted count of each state.
__global__ void boot_weights(int64_t ns, int64_t record_size, const int32_t *perm, const int32_t *state_orig,
                             const int32_t *mult, double *wgt, unsigned long long *omega)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ns; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t o = perm[i];
        const int32_t m = mult[o / record_size];
        wgt[i] = (double)m;
        if (m) atomicAdd(omega + state_orig[o], (unsigned long long)m);
    }
}

// Heat capacity C = beta^2 (<E^2> - <E>^2) and coverage <N> / n_sites per target
// (targets t = l n_mu + m, beta of row l).
__global__ void heat_cov(int nT, int nMu, const double *tbeta, const double *mean_n, const double *mean_e,
                         const double *mean_e2, double n_sites, double *heat, double *cov)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nT * nMu) return;
    const double b = tbeta[k / nMu];
    heat[k] = b * b * (mean_e2[k] - mean_e[k] * mean_e[k]);
    if (cov) cov[k] = mean_n[k] / n_sites;
}

// Standard deviation over B replicates of every target ([B][K] in, (B - 1) divisor).
__global__ void rep_sd(int B, int K, const double *rep, double *sd)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    double m = 0.0;
    for (int b = 0; b < B; ++b) m += rep[(size_t)b * K + k];
    m /= B;
    double v = 0.0;
    for (int b = 0; b < B; ++b) {
        const double d = rep[(size_t)b * K + k] - m;
        v += d * d;
    }
    sd[k] = sqrt(v / (double)(B - 1));
}

}  // namespace regc

using namespace regc;

struct regc_mbar {
    int L = 0, M = 0, S = 0, nN = 0;
    double lambda1 = 1.0;
    std::vector<double> t, mu, beta_l, lnz;
    hipStream_t stream = nullptr;
    DevBuf<double> beta_d, lnz_d, lnomega_d, f_d, fnew_d, logA_d, partial_d, delta_d, e_d, logd_d;
    DevBuf<int32_t> perm_d;           // sorted position -> original sample index
    DevBuf<uint32_t> obs_d;           // observables in sorted order [ns][n_obs]
    int n_obs = 0;
    DevBuf<int> chunk_n_d, chunk_b_d, chunk_e_d, seg_c0_d, seg_c1_d;
    int64_t ns = 0;
    int nchunks = 0;
    int gauge = -1;
    std::vector<double> lnomega;
    bool have_samples = false, solved = false;
    double ms_iter = 0.0;
    int64_t n_iter = 0;
    int method = 1, memory = 8;
    DevBuf<int32_t> n_orig_d, s_orig_d;   // N and state of the samples in the order given
    DevBuf<double> wgt_d;                 // bootstrap multiplicities in sorted order
    bool weighted = false;
};

static double lnz_of(double T, double mu, double lambda1)
{
    return mu / T - 3.0 * std::log(lambda1 / std::sqrt(T));
}

extern "C" int regc_mbar_create(const regc_grid *grid, double lambda1, int n_max, regc_mbar **out)
{
    REGC_CHECK(grid && out && grid->t && grid->mu, REGC_EINVAL, "null argument");
    REGC_CHECK(grid->n_t > 0 && grid->n_mu > 0 && n_max >= 0, REGC_EINVAL, "empty grid or negative n_max");
    REGC_CHECK(grid->n_t <= kMaxL, REGC_EUNSUPPORTED, "at most %d temperatures per reweighting grid", kMaxL);
    REGC_CHECK(n_max < 2048, REGC_EUNSUPPORTED, "n_max above 2047");
    REGC_CHECK(lambda1 > 0, REGC_EINVAL, "lambda1 must be positive");
    regc_mbar *mb = new regc_mbar();
    mb->L = grid->n_t; mb->M = grid->n_mu; mb->S = mb->L * mb->M; mb->nN = n_max + 1;
    mb->lambda1 = lambda1;
    mb->t.assign(grid->t, grid->t + mb->L);
    mb->mu.assign(grid->mu, grid->mu + mb->M);
    for (int l = 0; l < mb->L; ++l) {
        if (!(mb->t[l] > 0)) { delete mb; set_error("temperatures must be positive"); return REGC_EINVAL; }
        mb->beta_l.push_back(1.0 / mb->t[l]);
        for (int m = 0; m < mb->M; ++m) mb->lnz.push_back(lnz_of(mb->t[l], mb->mu[m], lambda1));
    }
    int rc;
    if ((rc = mb->beta_d.alloc(mb->L)) || (rc = mb->lnz_d.alloc(mb->S)) || (rc = mb->lnomega_d.alloc(mb->S)) ||
        (rc = mb->f_d.alloc(mb->S)) || (rc = mb->fnew_d.alloc(mb->S)) ||
        (rc = mb->logA_d.alloc((size_t)mb->L * mb->nN)) || (rc = mb->delta_d.alloc(1)) ||
        (rc = mb->seg_c0_d.alloc(mb->nN)) || (rc = mb->seg_c1_d.alloc(mb->nN))) {
        delete mb;
        return rc;
    }
    if (hipMemcpy(mb->beta_d.p, mb->beta_l.data(), sizeof(double) * mb->L, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(mb->lnz_d.p, mb->lnz.data(), sizeof(double) * mb->S, hipMemcpyHostToDevice) != hipSuccess) {
        delete mb;
        set_error("hipMemcpy failed");
        return REGC_EHIP;
    }
    *out = mb;
    return REGC_OK;
}

extern "C" int regc_mbar_set_stream(regc_mbar *mb, void *stream)
{
    REGC_CHECK(mb, REGC_EINVAL, "null handle");
    mb->stream = (hipStream_t)stream;
    return REGC_OK;
}

extern "C" int regc_mbar_set_samples(regc_mbar *mb, int64_t ns, const double *e, const int32_t *n,
                                     const int32_t *state, int on_device)
{
    REGC_CHECK(mb, REGC_EINVAL, "null handle");
    REGC_CHECK(ns > 0 && e && n && state, REGC_EINVAL, "no samples");
    REGC_CHECK(ns < (int64_t)1 << 31, REGC_EUNSUPPORTED, "more than 2^31 - 1 samples");
    // the handle's sample buffers are replaced below: until this call succeeds the
    // handle holds no samples (a failed call leaves it empty, not half updated)
    mb->have_samples = false;
    mb->solved = false;
    mb->n_obs = 0;
    hipStream_t s = mb->stream;
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    DevBuf<double> e_in;
    DevBuf<int32_t> &n_in = mb->n_orig_d, &s_in = mb->s_orig_d;
    DevBuf<int32_t> idx;
    mb->weighted = false;
    DevBuf<int32_t> &idx_out = mb->perm_d;
    DevBuf<uint32_t> keys, keys_out;
    DevBuf<unsigned long long> omega, seg;
    DevBuf<int> bad;
    int rc;
    if ((rc = e_in.alloc(ns)) || (rc = n_in.alloc(ns)) || (rc = s_in.alloc(ns)) || (rc = keys.alloc(ns)) ||
        (rc = keys_out.alloc(ns)) || (rc = idx.alloc(ns)) || (rc = idx_out.alloc(ns)) || (rc = omega.alloc(mb->S)) ||
        (rc = seg.alloc(mb->nN)) || (rc = bad.alloc(1)) || (rc = mb->e_d.alloc(ns)) || (rc = mb->logd_d.alloc(ns)))
        return rc;
    REGC_HIP(hipMemcpyAsync(e_in.p, e, sizeof(double) * ns, kind, s));
    REGC_HIP(hipMemcpyAsync(n_in.p, n, sizeof(int32_t) * ns, kind, s));
    REGC_HIP(hipMemcpyAsync(s_in.p, state, sizeof(int32_t) * ns, kind, s));
    REGC_HIP(hipMemsetAsync(omega.p, 0, sizeof(unsigned long long) * mb->S, s));
    REGC_HIP(hipMemsetAsync(seg.p, 0, sizeof(unsigned long long) * mb->nN, s));
    REGC_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), s));
    const int grid = (int)std::min<int64_t>((ns + 255) / 256, 4096);
    hipLaunchKernelGGL(mbar_count, dim3(grid), dim3(256), 0, s, ns, n_in.p, s_in.p, mb->nN, mb->S, omega.p, seg.p,
                       bad.p);
    REGC_HIP(hipGetLastError());
    int h_bad = 0;
    std::vector<unsigned long long> h_omega(mb->S), h_seg(mb->nN);
    REGC_HIP(hipMemcpyAsync(&h_bad, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
    REGC_HIP(hipMemcpyAsync(h_omega.data(), omega.p, sizeof(unsigned long long) * mb->S, hipMemcpyDeviceToHost, s));
    REGC_HIP(hipMemcpyAsync(h_seg.data(), seg.p, sizeof(unsigned long long) * mb->nN, hipMemcpyDeviceToHost, s));
    REGC_HIP(hipStreamSynchronize(s));
    REGC_CHECK(!h_bad, REGC_EINVAL, "sample with N outside 0..n_max or state outside the grid");

    // stable sort by N
    hipLaunchKernelGGL(mbar_iota_gather, dim3(grid), dim3(256), 0, s, ns, n_in.p, keys.p, idx.p);
    REGC_HIP(hipGetLastError());
    int end_bit = 1;
    while ((1 << end_bit) < mb->nN) ++end_bit;
    size_t temp_bytes = 0;
    REGC_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, temp_bytes, keys.p, keys_out.p, idx.p, idx_out.p, (int)ns, 0,
                                                end_bit, s));
    DevBuf<unsigned char> temp;
    if ((rc = temp.alloc(temp_bytes))) return rc;
    REGC_HIP(hipcub::DeviceRadixSort::SortPairs(temp.p, temp_bytes, keys.p, keys_out.p, idx.p, idx_out.p, (int)ns, 0,
                                                end_bit, s));
    hipLaunchKernelGGL(mbar_gather_e, dim3(grid), dim3(256), 0, s, ns, idx_out.p, e_in.p, mb->e_d.p);
    REGC_HIP(hipGetLastError());

    // chunks of one N each
    std::vector<int> cn, cb, ce, c0(mb->nN), c1(mb->nN);
    int64_t pos = 0;
    for (int N = 0; N < mb->nN; ++N) {
        c0[N] = (int)cn.size();
        const int64_t cnt = (int64_t)h_seg[N];
        for (int64_t k = 0; k < cnt; k += kChunk) {
            cn.push_back(N);
            cb.push_back((int)(pos + k));
            ce.push_back((int)(pos + std::min<int64_t>(cnt, k + kChunk)));
        }
        pos += cnt;
        c1[N] = (int)cn.size();
    }
    mb->nchunks = (int)cn.size();
    if ((rc = mb->chunk_n_d.alloc(mb->nchunks)) || (rc = mb->chunk_b_d.alloc(mb->nchunks)) ||
        (rc = mb->chunk_e_d.alloc(mb->nchunks)) || (rc = mb->partial_d.alloc((size_t)mb->nchunks * mb->L)))
        return rc;
    REGC_HIP(hipMemcpyAsync(mb->chunk_n_d.p, cn.data(), sizeof(int) * cn.size(), hipMemcpyHostToDevice, s));
    REGC_HIP(hipMemcpyAsync(mb->chunk_b_d.p, cb.data(), sizeof(int) * cb.size(), hipMemcpyHostToDevice, s));
    REGC_HIP(hipMemcpyAsync(mb->chunk_e_d.p, ce.data(), sizeof(int) * ce.size(), hipMemcpyHostToDevice, s));
    REGC_HIP(hipMemcpyAsync(mb->seg_c0_d.p, c0.data(), sizeof(int) * mb->nN, hipMemcpyHostToDevice, s));
    REGC_HIP(hipMemcpyAsync(mb->seg_c1_d.p, c1.data(), sizeof(int) * mb->nN, hipMemcpyHostToDevice, s));
    mb->lnomega.assign(mb->S, -INFINITY);
    mb->gauge = -1;
    for (int k = 0; k < mb->S; ++k)
        if (h_omega[k] > 0) {
            mb->lnomega[k] = std::log((double)h_omega[k]);
            if (mb->gauge < 0) mb->gauge = k;
        }
    REGC_HIP(hipMemcpyAsync(mb->lnomega_d.p, mb->lnomega.data(), sizeof(double) * mb->S, hipMemcpyHostToDevice, s));
    REGC_HIP(hipStreamSynchronize(s));
    mb->ns = ns;
    mb->have_samples = true;
    return REGC_OK;
}

static hipError_t launch_chunk(regc_mbar *mb, double *logd)
{
    const int L = mb->L;
    hipStream_t s = mb->stream;
#define CHUNK_CASE(LM, WT)                                                                                     \
    hipLaunchKernelGGL((mbar_chunk<LM, WT>), dim3(mb->nchunks), dim3(kMbarThreads), 0, s, L, mb->nN, mb->beta_d.p, \
                       mb->logA_d.p, mb->e_d.p, mb->chunk_n_d.p, mb->chunk_b_d.p, mb->chunk_e_d.p,               \
                       mb->partial_d.p, logd, mb->wgt_d.p)
    if (mb->weighted) {
        if (L <= 8) CHUNK_CASE(8, true);
        else if (L <= 16) CHUNK_CASE(16, true);
        else if (L <= 32) CHUNK_CASE(32, true);
        else CHUNK_CASE(64, true);
    } else {
        if (L <= 8) CHUNK_CASE(8, false);
        else if (L <= 16) CHUNK_CASE(16, false);
        else if (L <= 32) CHUNK_CASE(32, false);
        else CHUNK_CASE(64, false);
    }
#undef CHUNK_CASE
    return hipGetLastError();
}

static hipError_t mbar_iteration(regc_mbar *mb)
{
    hipStream_t s = mb->stream;
    hipLaunchKernelGGL(mbar_loga, dim3(mb->L), dim3(256), 0, s, mb->M, mb->nN, mb->lnomega_d.p, mb->f_d.p,
                       mb->lnz_d.p, mb->logA_d.p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = launch_chunk(mb, nullptr)) != hipSuccess) return e;
    hipLaunchKernelGGL(mbar_fnew, dim3(mb->L), dim3(256), sizeof(double) * mb->nN, s, mb->L, mb->M, mb->nN,
                       mb->partial_d.p, mb->seg_c0_d.p, mb->seg_c1_d.p, mb->logA_d.p, mb->lnz_d.p, mb->fnew_d.p);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(mbar_gauge, dim3(1), dim3(1024), 0, s, mb->S, mb->gauge, mb->lnomega_d.p, mb->fnew_d.p,
                       mb->f_d.p, mb->delta_d.p);
    return hipGetLastError();
}

// Least-squares coefficients gamma minimising || r - dR gamma ||_2 (dR: n x m,
// column-major) by modified Gram-Schmidt QR; columns that are numerically
// dependent on earlier ones get gamma = 0.
static void lsq_mgs(int n, int m, const std::vector<double> &dR, const std::vector<double> &r,
                    std::vector<double> &gamma)
{
    std::vector<double> Q(dR), R((size_t)m * m, 0.0), qtr(m, 0.0);
    std::vector<bool> keep(m, true);
    for (int j = 0; j < m; ++j) {
        double *qj = &Q[(size_t)j * n];
        double norm0 = 0.0;
        for (int i = 0; i < n; ++i) norm0 += qj[i] * qj[i];
        for (int k = 0; k < j; ++k) {
            if (!keep[k]) continue;
            const double *qk = &Q[(size_t)k * n];
            double d = 0.0;
            for (int i = 0; i < n; ++i) d += qk[i] * qj[i];
            R[(size_t)k * m + j] = d;
            for (int i = 0; i < n; ++i) qj[i] -= d * qk[i];
        }
        double nn = 0.0;
        for (int i = 0; i < n; ++i) nn += qj[i] * qj[i];
        if (nn <= 1e-24 * (norm0 + 1e-300)) {
            keep[j] = false;
            continue;
        }
        nn = std::sqrt(nn);
        R[(size_t)j * m + j] = nn;
        for (int i = 0; i < n; ++i) qj[i] /= nn;
        double d = 0.0;
        for (int i = 0; i < n; ++i) d += qj[i] * r[i];
        qtr[j] = d;
    }
    gamma.assign(m, 0.0);
    for (int j = m - 1; j >= 0; --j) {
        if (!keep[j]) continue;
        double v = qtr[j];
        for (int k = j + 1; k < m; ++k)
            if (keep[k]) v -= R[(size_t)j * m + k] * gamma[k];
        gamma[j] = v / R[(size_t)j * m + j];
    }
}

extern "C" int regc_mbar_set_solver(regc_mbar *mb, int method, int memory)
{
    REGC_CHECK(mb, REGC_EINVAL, "null handle");
    REGC_CHECK(method == 0 || method == 1, REGC_EINVAL, "method must be 0 (plain) or 1 (Anderson)");
    REGC_CHECK(memory >= 1 && memory <= 32, REGC_EINVAL, "memory must be 1..32");
    mb->method = method;
    mb->memory = memory;
    return REGC_OK;
}

// Fixed point f = g(f) of the self-consistent map (one device iteration = g plus the
// gauge).  Plain: f <- g(f).  Anderson acceleration (Walker & Ni, SIAM J. Numer.
// Anal. 49 (2011) 1715, type II) on the sampled states' components:
// x_{k+1} = g_k - dG gamma, gamma = argmin || r_k - dR gamma ||, r = g(x) - x, with
// at most min(memory, n - 2) differences for n sampled states (one component is
// fixed by the gauge, and more differences than free components make the least
// squares ill-posed).  A step that raises the residual tenfold restarts the history;
// a non-finite map value returns to the last finite one and takes plain steps for a
// while.  Converged when max |g(x) - x| over sampled states < tol.
// start: NULL (f = 0) or the starting iterate [S] (host).
static int solve_core(regc_mbar *mb, double tol, int max_iter, const double *start, int *iters, double *delta)
{
    hipStream_t s = mb->stream;
    if (start) REGC_HIP(hipMemcpyAsync(mb->f_d.p, start, sizeof(double) * mb->S, hipMemcpyHostToDevice, s));
    else REGC_HIP(hipMemsetAsync(mb->f_d.p, 0, sizeof(double) * mb->S, s));
    ScopedEvent e0, e1;
    REGC_HIP(e0.create());
    REGC_HIP(e1.create());
    REGC_HIP(hipEventRecord(e0.e, s));
    std::vector<int> idx;
    for (int k = 0; k < mb->S; ++k)
        if (mb->lnomega[k] != -INFINITY) idx.push_back(k);
    const int n = (int)idx.size();
    const int m = std::min(mb->memory, std::max(n - 2, 0));
    std::vector<double> x(mb->S, 0.0), gx(mb->S), xs(n), gs(n), r(n);
    if (start) x.assign(start, start + mb->S);
    std::deque<std::vector<double>> hist_r, hist_g;   // last residuals and map values (sampled part)
    double d = INFINITY, d_prev = INFINITY;
    int it = 0, plain_left = 0;
    bool conv = false;
    std::vector<double> good(mb->S, 0.0);            // the last finite map value
    const int check = mb->method == 0 ? 10 : 1;
    for (it = 0; it < max_iter;) {
        REGC_HIP(mbar_iteration(mb));   // f_d <- gauge(map(f_d)), delta_d <- max |new - old|
        ++it;
        if (it % check != 0 && it != max_iter) continue;
        REGC_HIP(hipMemcpyAsync(&d, mb->delta_d.p, sizeof(double), hipMemcpyDeviceToHost, s));
        if (mb->method == 1) REGC_HIP(hipMemcpyAsync(gx.data(), mb->f_d.p, sizeof(double) * mb->S, hipMemcpyDeviceToHost, s));
        REGC_HIP(hipStreamSynchronize(s));
        if (!(d <= 1e300)) {                        // NaN or inf
            if (mb->method == 0 || it == 1) break;  // nothing to return to: report it
            hist_r.clear();
            hist_g.clear();
            x = good;
            plain_left = 5;
            d_prev = INFINITY;
            REGC_HIP(hipMemcpyAsync(mb->f_d.p, x.data(), sizeof(double) * mb->S, hipMemcpyHostToDevice, s));
            continue;
        }
        if (d < tol) { conv = true; break; }
        if (mb->method == 0) continue;
        good = gx;
        for (int q = 0; q < n; ++q) {
            gs[q] = gx[idx[q]];
            r[q] = gx[idx[q]] - x[idx[q]];
        }
        if (d > 10.0 * d_prev) { hist_r.clear(); hist_g.clear(); }
        d_prev = d;
        hist_r.push_back(r);
        hist_g.push_back(gs);
        if ((int)hist_r.size() > m + 1) { hist_r.pop_front(); hist_g.pop_front(); }
        const int mk = (int)hist_r.size() - 1;
        std::vector<double> xn(gx);
        if (plain_left > 0) {
            --plain_left;
        } else if (mk > 0) {
            std::vector<double> dR((size_t)n * mk), gamma;
            for (int j = 0; j < mk; ++j)
                for (int q = 0; q < n; ++q) dR[(size_t)j * n + q] = hist_r[j + 1][q] - hist_r[j][q];
            lsq_mgs(n, mk, dR, r, gamma);
            for (int q = 0; q < n; ++q) {
                double v = gs[q];
                for (int j = 0; j < mk; ++j) v -= gamma[j] * (hist_g[j + 1][q] - hist_g[j][q]);
                xn[idx[q]] = v;
            }
        }
        x = xn;
        REGC_HIP(hipMemcpyAsync(mb->f_d.p, x.data(), sizeof(double) * mb->S, hipMemcpyHostToDevice, s));
    }
    REGC_HIP(hipEventRecord(e1.e, s));
    // f_d holds g of the last iterate; log D consistent with it
    hipLaunchKernelGGL(mbar_loga, dim3(mb->L), dim3(256), 0, s, mb->M, mb->nN, mb->lnomega_d.p, mb->f_d.p,
                       mb->lnz_d.p, mb->logA_d.p);
    REGC_HIP(hipGetLastError());
    REGC_HIP(launch_chunk(mb, mb->logd_d.p));
    REGC_HIP(hipStreamSynchronize(s));
    float ms = 0.f;
    REGC_HIP(hipEventElapsedTime(&ms, e0.e, e1.e));
    mb->ms_iter = ms;
    mb->n_iter = it;
    if (iters) *iters = it;
    if (delta) *delta = d;
    mb->solved = true;
    if (!conv) {
        set_error("reweighting did not converge: max |delta f| = %g after %d iterations", d, it);
        return REGC_ENOCONV;
    }
    return REGC_OK;
}

extern "C" int regc_mbar_solve(regc_mbar *mb, double tol, int max_iter, double *f_out, int *iters, double *delta)
{
    REGC_CHECK(mb, REGC_EINVAL, "null handle");
    REGC_CHECK(mb->have_samples, REGC_ESTATE, "no samples loaded");
    REGC_CHECK(max_iter > 0 && tol > 0, REGC_EINVAL, "max_iter and tol must be positive");
    const int rc = solve_core(mb, tol, max_iter, nullptr, iters, delta);
    if (rc != REGC_OK && rc != REGC_ENOCONV) return rc;
    if (f_out) REGC_HIP(hipMemcpy(f_out, mb->f_d.p, sizeof(double) * mb->S, hipMemcpyDeviceToHost));
    return rc;
}

// Target grid constants (beta per row, ln z per target) on the device.
struct TargetDev {
    int nT = 0, nMu = 0, nK = 0;
    DevBuf<double> tb_d, tz_d;
};

static int target_grid(regc_mbar *mb, const regc_grid *targets, TargetDev &T)
{
    T.nT = targets->n_t;
    T.nMu = targets->n_mu;
    T.nK = T.nT * T.nMu;
    REGC_CHECK(T.nT > 0 && T.nMu > 0, REGC_EINVAL, "empty target grid");
    std::vector<double> tb(T.nT), tz(T.nK);
    for (int l = 0; l < T.nT; ++l) {
        REGC_CHECK(targets->t[l] > 0, REGC_EINVAL, "target temperatures must be positive");
        tb[l] = 1.0 / targets->t[l];
        for (int m = 0; m < T.nMu; ++m) tz[l * T.nMu + m] = lnz_of(targets->t[l], targets->mu[m], mb->lambda1);
    }
    int rc;
    if ((rc = T.tb_d.alloc(T.nT)) || (rc = T.tz_d.alloc(T.nK))) return rc;
    REGC_HIP(hipMemcpyAsync(T.tb_d.p, tb.data(), sizeof(double) * T.nT, hipMemcpyHostToDevice, mb->stream));
    REGC_HIP(hipMemcpyAsync(T.tz_d.p, tz.data(), sizeof(double) * T.nK, hipMemcpyHostToDevice, mb->stream));
    return REGC_OK;
}

// Reweighted averages at the targets into device arrays (any may be NULL but mn).
static int targets_dev(regc_mbar *mb, const TargetDev &T, double *f, double *mn, double *me, double *me2,
                       double *pn, int32_t *ph)
{
    hipStream_t s = mb->stream;
    DevBuf<double> tpart;
    int rc;
    if ((rc = tpart.alloc((size_t)mb->nchunks * T.nT * 4))) return rc;
    hipLaunchKernelGGL(mbar_target_chunk, dim3(mb->nchunks), dim3(kMbarThreads), 0, s, T.nT, T.tb_d.p, mb->e_d.p,
                       mb->logd_d.p, mb->chunk_b_d.p, mb->chunk_e_d.p, tpart.p, mb->weighted ? mb->wgt_d.p : nullptr);
    REGC_HIP(hipGetLastError());
    hipLaunchKernelGGL(mbar_target_eval, dim3(T.nT), dim3(256), sizeof(double) * 3 * mb->nN, s, T.nT, T.nMu, mb->nN,
                       tpart.p, mb->seg_c0_d.p, mb->seg_c1_d.p, T.tz_d.p, f, mn, me, me2, pn, ph);
    REGC_HIP(hipGetLastError());
    REGC_HIP(hipStreamSynchronize(s));     // tpart is freed on return
    return REGC_OK;
}

extern "C" int regc_mbar_targets(regc_mbar *mb, const regc_grid *targets, double *f, double *mean_n,
                                 double *mean_e, double *mean_e2, double *p_n, int32_t *phase)
{
    REGC_CHECK(mb && targets && mean_n && targets->t && targets->mu, REGC_EINVAL, "null argument");
    REGC_CHECK(mb->solved, REGC_ESTATE, "solve first");
    TargetDev T;
    int rc;
    if ((rc = target_grid(mb, targets, T))) return rc;
    const int nK = T.nK;
    DevBuf<double> f_d, mn_d, me_d, me2_d, pn_d;
    DevBuf<int32_t> ph_d;
    if ((rc = f_d.alloc(nK)) || (rc = mn_d.alloc(nK)) || (rc = me_d.alloc(nK)) || (rc = me2_d.alloc(nK)) ||
        (rc = ph_d.alloc(nK)) || (rc = pn_d.alloc(p_n ? (size_t)nK * mb->nN : 1)))
        return rc;
    if ((rc = targets_dev(mb, T, f_d.p, mn_d.p, me_d.p, me2_d.p, p_n ? pn_d.p : nullptr, ph_d.p))) return rc;
    if (f) REGC_HIP(hipMemcpy(f, f_d.p, sizeof(double) * nK, hipMemcpyDeviceToHost));
    REGC_HIP(hipMemcpy(mean_n, mn_d.p, sizeof(double) * nK, hipMemcpyDeviceToHost));
    if (mean_e) REGC_HIP(hipMemcpy(mean_e, me_d.p, sizeof(double) * nK, hipMemcpyDeviceToHost));
    if (mean_e2) REGC_HIP(hipMemcpy(mean_e2, me2_d.p, sizeof(double) * nK, hipMemcpyDeviceToHost));
    if (phase) REGC_HIP(hipMemcpy(phase, ph_d.p, sizeof(int32_t) * nK, hipMemcpyDeviceToHost));
    if (p_n) REGC_HIP(hipMemcpy(p_n, pn_d.p, sizeof(double) * nK * mb->nN, hipMemcpyDeviceToHost));
    return REGC_OK;
}

// ---- reweighted averages without allocation ----
// Device scratch of regc_mbar_targets_static: the target constants, the per-chunk
// partial sums and the outputs before their copy to the host.  Every GPU the library
// runs on holds its own copy for the life of the process; host code reaches it only
// through the address hipGetSymbolAddress returns on that device.
constexpr size_t kStaticScratchDoubles = (size_t)1 << 19;     // 4 MiB
constexpr int kStaticMaxT = 1024, kStaticMaxK = 4096;
constexpr int kStaticMaxDevices = 64;
static __device__ __align__(256) double scratch[kStaticScratchDoubles];
static std::mutex g_static_mu;
static double *g_static_ptr[kStaticMaxDevices];

// The current device's scratch address (looked up once per device, with it current).
static int static_scratch(double **out)
{
    int dev = -1;
    REGC_HIP(hipGetDevice(&dev));
    REGC_CHECK(dev >= 0 && dev < kStaticMaxDevices, REGC_EINVAL, "device %d beyond the static scratch table", dev);
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[dev]) {
        void *p = nullptr;
        REGC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        REGC_CHECK(p != nullptr, REGC_EINVAL, "no address for the static scratch on device %d", dev);
        g_static_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_static_ptr[dev];
    return REGC_OK;
}

extern "C" int regc_mbar_targets_static(regc_mbar *mb, const regc_grid *targets, double *f, double *mean_n,
                                        double *mean_e, double *mean_e2, int32_t *phase)
{
    REGC_CHECK(mb && targets && mean_n && targets->t && targets->mu, REGC_EINVAL, "null argument");
    REGC_CHECK(mb->solved, REGC_ESTATE, "solve first");
    const int nT = targets->n_t, nMu = targets->n_mu;
    REGC_CHECK(nT > 0 && nMu > 0, REGC_EINVAL, "empty target grid");
    REGC_CHECK(nT <= kStaticMaxT && (int64_t)nT * nMu <= kStaticMaxK, REGC_EINVAL,
               "target grid %d x %d beyond the static limits (%d temperatures, %d targets)", nT, nMu, kStaticMaxT,
               kStaticMaxK);
    const int nK = nT * nMu;
    // scratch: tb [nT] | tz [nK] | partials [nchunks][nT][4] | f, mean_n, mean_e, mean_e2, phase [nK] each
    const size_t need = (size_t)nT + (size_t)nK + (size_t)mb->nchunks * nT * 4 + (size_t)5 * nK;
    REGC_CHECK(need <= kStaticScratchDoubles, REGC_EINVAL,
               "%zu doubles of scratch needed (%d sample chunks x %d temperatures), %zu available", need,
               mb->nchunks, nT, kStaticScratchDoubles);
    double tb[kStaticMaxT], tz[kStaticMaxK];
    for (int l = 0; l < nT; ++l) {
        REGC_CHECK(targets->t[l] > 0, REGC_EINVAL, "target temperatures must be positive");
        tb[l] = 1.0 / targets->t[l];
        for (int m = 0; m < nMu; ++m) tz[l * nMu + m] = lnz_of(targets->t[l], targets->mu[m], mb->lambda1);
    }
    double *sp = nullptr;
    int rc;
    if ((rc = static_scratch(&sp))) return rc;
    double *tb_d = sp, *tz_d = tb_d + nT, *part = tz_d + nK, *f_d = part + (size_t)mb->nchunks * nT * 4;
    double *mn_d = f_d + nK, *me_d = mn_d + nK, *me2_d = me_d + nK;
    int32_t *ph_d = reinterpret_cast<int32_t *>(me2_d + nK);
    hipStream_t s = mb->stream;
    REGC_HIP(hipMemcpyAsync(tb_d, tb, sizeof(double) * nT, hipMemcpyHostToDevice, s));
    REGC_HIP(hipMemcpyAsync(tz_d, tz, sizeof(double) * nK, hipMemcpyHostToDevice, s));
    // every partial and output entry read below is written by these two kernels
    hipLaunchKernelGGL(mbar_target_chunk, dim3(mb->nchunks), dim3(kMbarThreads), 0, s, nT, tb_d, mb->e_d.p,
                       mb->logd_d.p, mb->chunk_b_d.p, mb->chunk_e_d.p, part, mb->weighted ? mb->wgt_d.p : nullptr);
    REGC_HIP(hipGetLastError());
    hipLaunchKernelGGL(mbar_target_eval, dim3(nT), dim3(256), sizeof(double) * 3 * mb->nN, s, nT, nMu, mb->nN, part,
                       mb->seg_c0_d.p, mb->seg_c1_d.p, tz_d, f_d, mn_d, me_d, me2_d, nullptr, ph_d);
    REGC_HIP(hipGetLastError());
    if (f) REGC_HIP(hipMemcpyAsync(f, f_d, sizeof(double) * nK, hipMemcpyDeviceToHost, s));
    REGC_HIP(hipMemcpyAsync(mean_n, mn_d, sizeof(double) * nK, hipMemcpyDeviceToHost, s));
    if (mean_e) REGC_HIP(hipMemcpyAsync(mean_e, me_d, sizeof(double) * nK, hipMemcpyDeviceToHost, s));
    if (mean_e2) REGC_HIP(hipMemcpyAsync(mean_e2, me2_d, sizeof(double) * nK, hipMemcpyDeviceToHost, s));
    if (phase) REGC_HIP(hipMemcpyAsync(phase, ph_d, sizeof(int32_t) * nK, hipMemcpyDeviceToHost, s));
    REGC_HIP(hipStreamSynchronize(s));     // the stack copies of tb, tz live until here
    return REGC_OK;
}

extern "C" int regc_mbar_set_observables(regc_mbar *mb, const uint32_t *obs, int n_obs, int on_device)
{
    REGC_CHECK(mb && obs, REGC_EINVAL, "null argument");
    REGC_CHECK(mb->have_samples, REGC_ESTATE, "set the samples first");
    REGC_CHECK(n_obs > 0 && n_obs <= 4096, REGC_EINVAL, "n_obs must be 1..4096");
    mb->n_obs = 0;     // no observables until this call succeeds
    hipStream_t s = mb->stream;
    const size_t count = (size_t)mb->ns * n_obs;
    DevBuf<uint32_t> in;
    int rc;
    if ((rc = in.alloc(count)) || (rc = mb->obs_d.alloc(count))) return rc;
    REGC_HIP(hipMemcpyAsync(in.p, obs, sizeof(uint32_t) * count,
                            on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    const int grid = (int)std::min<size_t>((count + 255) / 256, 8192);
    hipLaunchKernelGGL(mbar_gather_obs, dim3(grid), dim3(256), 0, s, (int64_t)mb->ns, n_obs, mb->perm_d.p, in.p,
                       mb->obs_d.p);
    REGC_HIP(hipGetLastError());
    REGC_HIP(hipStreamSynchronize(s));
    mb->n_obs = n_obs;
    return REGC_OK;
}

extern "C" int regc_mbar_observables(regc_mbar *mb, const regc_grid *targets, double *mean, double *cond)
{
    REGC_CHECK(mb && targets && targets->t && targets->mu, REGC_EINVAL, "null argument");
    REGC_CHECK(mb->solved, REGC_ESTATE, "solve first");
    REGC_CHECK(mb->n_obs > 0, REGC_ESTATE, "no observables loaded");
    REGC_CHECK(!mb->weighted, REGC_ESTATE, "a bootstrap is in progress");
    const int nT = targets->n_t, nMu = targets->n_mu, nK = nT * nMu, no = mb->n_obs;
    REGC_CHECK(nT > 0 && nMu > 0, REGC_EINVAL, "empty target grid");
    std::vector<double> tb(nT), tz(nK);
    for (int l = 0; l < nT; ++l) {
        REGC_CHECK(targets->t[l] > 0, REGC_EINVAL, "target temperatures must be positive");
        tb[l] = 1.0 / targets->t[l];
        for (int m = 0; m < nMu; ++m) tz[l * nMu + m] = lnz_of(targets->t[l], targets->mu[m], mb->lambda1);
    }
    hipStream_t s = mb->stream;
    DevBuf<double> tb_d, tz_d, part, cond_d, mean_d;
    int rc;
    if ((rc = tb_d.alloc(nT)) || (rc = tz_d.alloc(nK)) || (rc = part.alloc((size_t)mb->nchunks * nT * (no + 2))) ||
        (rc = cond_d.alloc((size_t)nT * mb->nN * no)) || (rc = mean_d.alloc(mean ? (size_t)nK * no : 1)))
        return rc;
    REGC_HIP(hipMemcpyAsync(tb_d.p, tb.data(), sizeof(double) * nT, hipMemcpyHostToDevice, s));
    REGC_HIP(hipMemcpyAsync(tz_d.p, tz.data(), sizeof(double) * nK, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(mbar_obs_chunk, dim3(mb->nchunks, nT), dim3(kMbarThreads), 0, s, nT, no, tb_d.p, mb->e_d.p,
                       mb->logd_d.p, mb->chunk_b_d.p, mb->chunk_e_d.p, mb->obs_d.p, part.p);
    REGC_HIP(hipGetLastError());
    hipLaunchKernelGGL(mbar_obs_eval, dim3(nT), dim3(256), 2 * sizeof(double) * mb->nN, s, nT, nMu, mb->nN, no,
                       part.p, mb->seg_c0_d.p, mb->seg_c1_d.p, tz_d.p, cond_d.p, mean ? mean_d.p : nullptr);
    REGC_HIP(hipGetLastError());
    REGC_HIP(hipStreamSynchronize(s));
    if (cond) REGC_HIP(hipMemcpy(cond, cond_d.p, sizeof(double) * (size_t)nT * mb->nN * no, hipMemcpyDeviceToHost));
    if (mean) REGC_HIP(hipMemcpy(mean, mean_d.p, sizeof(double) * (size_t)nK * no, hipMemcpyDeviceToHost));
    return REGC_OK;
}

extern "C" int regc_mbar_timing(regc_mbar *mb, double *ms_iter_total, int64_t *n_iter)
{
    REGC_CHECK(mb, REGC_EINVAL, "null handle");
    if (ms_iter_total) *ms_iter_total = mb->ms_iter;
    if (n_iter) *n_iter = mb->n_iter;
    return REGC_OK;
}

extern "C" void regc_mbar_destroy(regc_mbar *mb) { delete mb; }

// ---------------------------------------------------------------------------
// Estimates with their errors: the solve, the averages at the targets, batch means
// at the sampled states and a moving-block bootstrap over records (re-solving with
// the records' multiplicities as sample weights, warm-started from the full solve).
extern "C" void regc_default_reweight_opts(regc_reweight_opts *o)
{
    if (!o) return;
    o->n_batches = 20;
    o->n_boot = 100;
    o->record_size = 0;
    o->block_records = 0;
    o->seed = 1;
    o->n_sites = 0.0;
}

// Sets the handle's state counts (and gauge) from a device array of counts.
static int set_omega(regc_mbar *mb, const unsigned long long *omega_d)
{
    std::vector<unsigned long long> h(mb->S);
    REGC_HIP(hipMemcpyAsync(h.data(), omega_d, sizeof(unsigned long long) * mb->S, hipMemcpyDeviceToHost, mb->stream));
    REGC_HIP(hipStreamSynchronize(mb->stream));
    mb->lnomega.assign(mb->S, -INFINITY);
    mb->gauge = -1;
    for (int k = 0; k < mb->S; ++k)
        if (h[k] > 0) {
            mb->lnomega[k] = std::log((double)h[k]);
            if (mb->gauge < 0) mb->gauge = k;
        }
    REGC_HIP(hipMemcpyAsync(mb->lnomega_d.p, mb->lnomega.data(), sizeof(double) * mb->S, hipMemcpyHostToDevice,
                            mb->stream));
    return REGC_OK;
}

// log D of the current f (after changing the weights or restoring f)
static int refresh_logd(regc_mbar *mb)
{
    hipLaunchKernelGGL(mbar_loga, dim3(mb->L), dim3(256), 0, mb->stream, mb->M, mb->nN, mb->lnomega_d.p, mb->f_d.p,
                       mb->lnz_d.p, mb->logA_d.p);
    REGC_HIP(hipGetLastError());
    REGC_HIP(launch_chunk(mb, mb->logd_d.p));
    return REGC_OK;
}

// Per-state mean of N and its batch-means SE of ns samples (state, n) in the order
// given, device arrays; outputs device arrays [S].  EINVAL on a state outside 0..S-1
// or a negative N.
static int batch_means_dev(hipStream_t s, int64_t ns, const int32_t *st_d, const int32_t *n_d, int S, int B,
                           double *mean_d, double *se_d)
{
    DevBuf<uint32_t> keys, keys_out;
    DevBuf<int32_t> idx, idx_out;
    DevBuf<int64_t> start_d, count_d;
    DevBuf<unsigned long long> bsum, bcnt;
    DevBuf<int> bad;
    int rc;
    if ((rc = keys.alloc(ns)) || (rc = keys_out.alloc(ns)) || (rc = idx.alloc(ns)) || (rc = idx_out.alloc(ns)) ||
        (rc = start_d.alloc(S)) || (rc = count_d.alloc(S)) || (rc = bsum.alloc((size_t)S * B)) ||
        (rc = bcnt.alloc((size_t)S * B)) || (rc = bad.alloc(1)))
        return rc;
    const int grid = (int)std::min<int64_t>((ns + 255) / 256, 4096);
    // the inputs are checked before they are used as sort keys
    int h_bad = 0;
    hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, s, (int64_t)1, 0, bad.p);
    hipLaunchKernelGGL(bm_check, dim3(grid), dim3(256), 0, s, ns, st_d, n_d, S, bad.p);
    REGC_HIP(hipGetLastError());
    REGC_HIP(hipMemcpyAsync(&h_bad, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
    REGC_HIP(hipStreamSynchronize(s));
    REGC_CHECK(!h_bad, REGC_EINVAL, "a sample's state is outside 0..%d or its N is negative", S - 1);
    // stable sort of the sample indices by state: each state's series in sample order
    hipLaunchKernelGGL(mbar_iota_gather, dim3(grid), dim3(256), 0, s, ns, st_d, keys.p, idx.p);
    REGC_HIP(hipGetLastError());
    int end_bit = 1;
    while ((1 << end_bit) < S) ++end_bit;
    size_t temp_bytes = 0;
    REGC_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, temp_bytes, keys.p, keys_out.p, idx.p, idx_out.p, (int)ns, 0,
                                                end_bit, s));
    DevBuf<unsigned char> temp;
    if ((rc = temp.alloc(temp_bytes))) return rc;
    REGC_HIP(hipcub::DeviceRadixSort::SortPairs(temp.p, temp_bytes, keys.p, keys_out.p, idx.p, idx_out.p, (int)ns, 0,
                                                end_bit, s));
    hipLaunchKernelGGL(bm_bounds, dim3((S + 255) / 256), dim3(256), 0, s, ns, S, keys_out.p, start_d.p, count_d.p);
    REGC_HIP(hipGetLastError());
    hipLaunchKernelGGL(bm_segments, dim3(S * B), dim3(256), 0, s, B, idx_out.p, n_d, start_d.p, count_d.p, bsum.p,
                       bcnt.p);
    REGC_HIP(hipGetLastError());
    hipLaunchKernelGGL(bm_finish, dim3((S + 255) / 256), dim3(256), 0, s, S, B, bsum.p, bcnt.p, count_d.p, mean_d,
                       se_d);
    REGC_HIP(hipGetLastError());
    REGC_HIP(hipStreamSynchronize(s));
    return REGC_OK;
}

extern "C" int regc_batch_means(int64_t ns, const int32_t *state, const int32_t *n, int n_states, int n_batches,
                                int on_device, double *mean, double *se, void *stream)
{
    REGC_CHECK(state && n && mean && se, REGC_EINVAL, "null argument");
    REGC_CHECK(ns > 0 && ns <= INT32_MAX, REGC_EINVAL, "sample count must be 1..2^31-1");
    REGC_CHECK(n_states > 0 && n_batches >= 2, REGC_EINVAL, "n_states must be positive and n_batches >= 2");
    hipStream_t s = static_cast<hipStream_t>(stream);
    DevBuf<int32_t> st_in, n_in;
    DevBuf<double> m_d, se_d;
    int rc;
    if ((rc = m_d.alloc(n_states)) || (rc = se_d.alloc(n_states))) return rc;
    const int32_t *st_d = state, *n_d = n;
    if (!on_device) {
        if ((rc = st_in.alloc(ns)) || (rc = n_in.alloc(ns))) return rc;
        REGC_HIP(hipMemcpyAsync(st_in.p, state, sizeof(int32_t) * ns, hipMemcpyHostToDevice, s));
        REGC_HIP(hipMemcpyAsync(n_in.p, n, sizeof(int32_t) * ns, hipMemcpyHostToDevice, s));
        st_d = st_in.p;
        n_d = n_in.p;
    }
    if ((rc = batch_means_dev(s, ns, st_d, n_d, n_states, n_batches, m_d.p, se_d.p))) return rc;
    REGC_HIP(hipMemcpy(mean, m_d.p, sizeof(double) * n_states, hipMemcpyDeviceToHost));
    REGC_HIP(hipMemcpy(se, se_d.p, sizeof(double) * n_states, hipMemcpyDeviceToHost));
    return REGC_OK;
}

extern "C" int regc_reweight(regc_mbar *mb, const regc_grid *targets, double tol, int max_iter,
                             const regc_reweight_opts *opts, double *f_states, double *mean_state_n,
                             double *se_state_n, double *mean_n, double *se_n, int32_t *phase, double *coverage,
                             double *se_coverage, double *heat_cap, double *se_heat_cap, double *p_n)
{
    REGC_CHECK(mb && targets && targets->t && targets->mu, REGC_EINVAL, "null argument");
    REGC_CHECK(mb->have_samples, REGC_ESTATE, "no samples loaded");
    REGC_CHECK(max_iter > 0 && tol > 0, REGC_EINVAL, "max_iter and tol must be positive");
    regc_reweight_opts o;
    regc_default_reweight_opts(&o);
    if (opts) o = *opts;
    const int64_t rs = o.record_size > 0 ? o.record_size : mb->S;
    REGC_CHECK(o.n_batches >= 2 && o.n_boot >= 0 && o.n_boot != 1, REGC_EINVAL,
               "n_batches must be >= 2 and n_boot 0 or >= 2");
    REGC_CHECK(mb->ns % rs == 0, REGC_EINVAL, "%lld samples are not whole records of %lld", (long long)mb->ns,
               (long long)rs);
    const int64_t R = mb->ns / rs;
    const int64_t blk = o.block_records > 0 ? o.block_records : std::max<int64_t>(1, R / o.n_batches);
    REGC_CHECK(blk <= R, REGC_EINVAL, "bootstrap blocks of %lld records exceed the %lld records", (long long)blk,
               (long long)R);
    REGC_CHECK((coverage == nullptr && se_coverage == nullptr) || o.n_sites > 0, REGC_EINVAL,
               "coverage needs n_sites > 0");
    hipStream_t s = mb->stream;
    mb->weighted = false;
    int rc = solve_core(mb, tol, max_iter, nullptr, nullptr, nullptr);
    if (rc != REGC_OK && rc != REGC_ENOCONV) return rc;
    const int solve_rc = rc;
    std::vector<double> f0(mb->S);
    REGC_HIP(hipMemcpy(f0.data(), mb->f_d.p, sizeof(double) * mb->S, hipMemcpyDeviceToHost));
    if (f_states) std::copy(f0.begin(), f0.end(), f_states);
    TargetDev T;
    if ((rc = target_grid(mb, targets, T))) return rc;
    const int nK = T.nK;
    DevBuf<double> mn, me, me2, pn, heat, cov, smean, sse;
    DevBuf<int32_t> ph;
    if ((rc = mn.alloc(nK)) || (rc = me.alloc(nK)) || (rc = me2.alloc(nK)) || (rc = ph.alloc(nK)) ||
        (rc = pn.alloc(p_n ? (size_t)nK * mb->nN : 1)) || (rc = heat.alloc(nK)) || (rc = cov.alloc(nK)) ||
        (rc = smean.alloc(mb->S)) || (rc = sse.alloc(mb->S)))
        return rc;
    if ((rc = targets_dev(mb, T, nullptr, mn.p, me.p, me2.p, p_n ? pn.p : nullptr, ph.p))) return rc;
    hipLaunchKernelGGL(heat_cov, dim3((nK + 255) / 256), dim3(256), 0, s, T.nT, T.nMu, T.tb_d.p, mn.p, me.p, me2.p,
                       o.n_sites > 0 ? o.n_sites : 1.0, heat.p, cov.p);
    REGC_HIP(hipGetLastError());
    if ((rc = batch_means_dev(mb->stream, mb->ns, mb->s_orig_d.p, mb->n_orig_d.p, mb->S, o.n_batches, smean.p,
                              sse.p)))
        return rc;
    REGC_HIP(hipStreamSynchronize(s));
    if (mean_n) REGC_HIP(hipMemcpy(mean_n, mn.p, sizeof(double) * nK, hipMemcpyDeviceToHost));
    if (phase) REGC_HIP(hipMemcpy(phase, ph.p, sizeof(int32_t) * nK, hipMemcpyDeviceToHost));
    if (p_n) REGC_HIP(hipMemcpy(p_n, pn.p, sizeof(double) * nK * mb->nN, hipMemcpyDeviceToHost));
    if (heat_cap) REGC_HIP(hipMemcpy(heat_cap, heat.p, sizeof(double) * nK, hipMemcpyDeviceToHost));
    if (coverage) REGC_HIP(hipMemcpy(coverage, cov.p, sizeof(double) * nK, hipMemcpyDeviceToHost));
    if (mean_state_n) REGC_HIP(hipMemcpy(mean_state_n, smean.p, sizeof(double) * mb->S, hipMemcpyDeviceToHost));
    if (se_state_n) REGC_HIP(hipMemcpy(se_state_n, sse.p, sizeof(double) * mb->S, hipMemcpyDeviceToHost));
    const bool want_boot = se_n || se_coverage || se_heat_cap;
    if (!want_boot || o.n_boot == 0) {
        const double nan = NAN;
        for (int k = 0; k < nK; ++k) {
            if (se_n) se_n[k] = nan;
            if (se_coverage) se_coverage[k] = nan;
            if (se_heat_cap) se_heat_cap[k] = nan;
        }
        return solve_rc;
    }
    // bootstrap replicates
    const int B = o.n_boot;
    const std::vector<double> lnomega0 = mb->lnomega;
    const int gauge0 = mb->gauge;
    DevBuf<int32_t> mult;
    DevBuf<unsigned long long> omega;
    DevBuf<double> rep_n, rep_c, sd_n, sd_c, bme, bme2;
    if ((rc = mult.alloc(R)) || (rc = omega.alloc(mb->S)) || (rc = mb->wgt_d.alloc(mb->ns)) ||
        (rc = rep_n.alloc((size_t)B * nK)) || (rc = rep_c.alloc((size_t)B * nK)) || (rc = sd_n.alloc(nK)) ||
        (rc = sd_c.alloc(nK)) || (rc = bme.alloc(nK)) || (rc = bme2.alloc(nK)))
        return rc;
    const int grid = (int)std::min<int64_t>((mb->ns + 255) / 256, 4096);
    const int64_t nblk = (R + blk - 1) / blk;
    int boot_rc = REGC_OK;
    for (int b = 0; b < B && boot_rc == REGC_OK; ++b) {
        hipLaunchKernelGGL(fill_i32, dim3((unsigned)std::min<int64_t>((R + 255) / 256, 4096)), dim3(256), 0, s, R, 0,
                           mult.p);
        hipLaunchKernelGGL(boot_mult, dim3((unsigned)std::min<int64_t>((nblk + 255) / 256, 4096)), dim3(256), 0, s, R,
                           blk, b, (uint32_t)o.seed, (uint32_t)(o.seed >> 32), mult.p);
        hipLaunchKernelGGL(fill_u64, dim3(1), dim3(256), 0, s, (int64_t)mb->S, omega.p);
        hipLaunchKernelGGL(boot_weights, dim3(grid), dim3(256), 0, s, mb->ns, rs, mb->perm_d.p, mb->s_orig_d.p, mult.p,
                           mb->wgt_d.p, omega.p);
        REGC_HIP(hipGetLastError());
        if ((rc = set_omega(mb, omega.p))) { boot_rc = rc; break; }
        mb->weighted = true;
        rc = solve_core(mb, tol, max_iter, f0.data(), nullptr, nullptr);
        if (rc != REGC_OK && rc != REGC_ENOCONV) { boot_rc = rc; break; }
        if (rc == REGC_ENOCONV) boot_rc = REGC_ENOCONV;
        if ((rc = targets_dev(mb, T, nullptr, rep_n.p + (size_t)b * nK, bme.p, bme2.p, nullptr, ph.p))) {
            boot_rc = rc;
            break;
        }
        hipLaunchKernelGGL(heat_cov, dim3((nK + 255) / 256), dim3(256), 0, s, T.nT, T.nMu, T.tb_d.p,
                           rep_n.p + (size_t)b * nK, bme.p, bme2.p, 1.0, rep_c.p + (size_t)b * nK, nullptr);
        REGC_HIP(hipGetLastError());
    }
    // back to the full data: counts, f, log D
    mb->weighted = false;
    mb->lnomega = lnomega0;
    mb->gauge = gauge0;
    REGC_HIP(hipMemcpyAsync(mb->lnomega_d.p, lnomega0.data(), sizeof(double) * mb->S, hipMemcpyHostToDevice, s));
    REGC_HIP(hipMemcpyAsync(mb->f_d.p, f0.data(), sizeof(double) * mb->S, hipMemcpyHostToDevice, s));
    if ((rc = refresh_logd(mb))) return rc;
    REGC_HIP(hipStreamSynchronize(s));
    if (boot_rc != REGC_OK && boot_rc != REGC_ENOCONV) return boot_rc;
    hipLaunchKernelGGL(rep_sd, dim3((nK + 255) / 256), dim3(256), 0, s, B, nK, rep_n.p, sd_n.p);
    hipLaunchKernelGGL(rep_sd, dim3((nK + 255) / 256), dim3(256), 0, s, B, nK, rep_c.p, sd_c.p);
    REGC_HIP(hipGetLastError());
    REGC_HIP(hipStreamSynchronize(s));
    std::vector<double> h(nK);
    REGC_HIP(hipMemcpy(h.data(), sd_n.p, sizeof(double) * nK, hipMemcpyDeviceToHost));
    if (se_n) std::copy(h.begin(), h.end(), se_n);
    if (se_coverage)
        for (int k = 0; k < nK; ++k) se_coverage[k] = h[k] / o.n_sites;
    if (se_heat_cap) REGC_HIP(hipMemcpy(se_heat_cap, sd_c.p, sizeof(double) * nK, hipMemcpyDeviceToHost));
    if (boot_rc == REGC_ENOCONV) {
        set_error("a bootstrap replicate did not converge");
        return REGC_ENOCONV;
    }
    return solve_rc;
}
