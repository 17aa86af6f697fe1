// learned.hip -- REGC sweeps with the learned insertion proposal (an extension
// of the method, not in the paper): one walker per workgroup of four wavefronts,
// the walker's gas, voxel occupancy and the network's output held in LDS for the
// whole launch, the network evaluated inside the trial loop.
//
// Proposal (mixture, so that its density never vanishes): an insertion point is a
// voxel v drawn from the network's categorical P(v | occ(X)) plus a uniform offset
// inside the voxel with probability alpha (word B3 of the trial), else a uniform
// point of V.  Density q(r|X) = alpha P(v(r)|occ(X)) / V_vox + (1 - alpha) / V;
// with Lq = ln(q V) = ln(1 + alpha (4096 P - 1)) the acceptance ratios of Eqs. (2)
// and (3) (Sec. II.A.1) become
//   insertion  ln A = ln z + ln V - ln(N+1) - Lq(r | X)        - beta dE,
//   removal    ln A = ln N - ln z - ln V    + Lq(r_i | X \ i)  - beta dE,
// which leaves Eq. (1) the stationary law for any network.  A voxel is drawn by
// Gumbel-max (FP64 build: argmax_v logit_v - ln(-ln u_v), u_v from Philox block
// (trial, sweep, walker, 16 + v/4), word v%4; the 32-bit u_v make each voxel's
// probability the softmax up to their discreteness) or by inverse CDF with one
// 53-bit uniform from words x, y of block (trial, sweep, walker, 16) over FP32
// weights summed in FP64 (FP32 build), whose probabilities the acceptance uses.
//
// Per trial: the same Philox words as the plain sweep kernel (displacement and the
// uniform branch give the plain trajectories); for insertions and removals the
// network runs on the ascending list of occupied voxels (first layer: sum of
// count x W1 row).  FP32 build: layers 2-4 on v_mfma_f32_16x16x16_bf16 with the
// activation vector as every row of A, log-normaliser and the inverse-CDF draw in
// FP32.
// FP64 (parity) build: layers 2-4 as sequential FP32 sums of exact bfloat16
// products, GELU's erf in FP64, log-normaliser and Gumbel keys in FP64, so the
// network output is the oracle's bit for bit and trajectories can be compared
// trial by trial.  The 4096 logits of the current occupancy stay in LDS and serve
// later insertions until the occupancy changes.  The energy change is split over
// the four waves and combined through LDS in a fixed order.
#include "sweep_dev.h"
#include "learn_dev.h"
#include "mlp_dev.h"

#if defined(REGC_FP64)
#define LEARNED_LAUNCH launch_learned_f64
#define NET_EVAL_LAUNCH launch_net_eval_f64
#else
#define LEARNED_LAUNCH launch_learned_f32
#define NET_EVAL_LAUNCH launch_net_eval_f32
#endif

namespace regc {
namespace REGC_PREC {

using mlpk::bf16;
using mlpk::bf16x4;
using mlpk::f32x4;
using mlpk::bf2f;
using mlpk::f2bf;
using mlpk::gelu;

constexpr int kLT = kWave * kLearnWaves;   // threads per walker

struct Grid {
    double gx, gy, gz, zlo;      // cells per unit length, bottom of the gas region
    double cx, cy, cz;           // cell widths
};

// voxel (iz*16 + iy)*16 + ix of a point, indices clamped to the grid
__device__ __forceinline__ int voxel_of(const Grid &g, double x, double y, double z)
{
    int ix = (int)floor(x * g.gx), iy = (int)floor(y * g.gy), iz = (int)floor((z - g.zlo) * g.gz);
    ix = ix < 0 ? 0 : (ix > kNetGrid - 1 ? kNetGrid - 1 : ix);
    iy = iy < 0 ? 0 : (iy > kNetGrid - 1 ? kNetGrid - 1 : iy);
    iz = iz < 0 ? 0 : (iz > kNetGrid - 1 ? kNetGrid - 1 : iz);
    return (iz * kNetGrid + iy) * kNetGrid + ix;
}

#if defined(REGC_FP64)
// parity build: the network's arithmetic is the oracle's, bit for bit -- sequential
// FP32 sums of exact bfloat16 products in ascending k, GELU with erf in FP64 --
// and the log-normaliser and Gumbel keys are FP64
constexpr bool kExact = true;
#else
// production build: layers 2-4 on MFMA, log-normaliser and Gumbel keys in FP32
constexpr bool kExact = false;
#endif

// GELU with erf evaluated in FP64 and the rest in FP32 (1.4142135623730951 is the
// double nearest sqrt 2)
__device__ __forceinline__ float gelu_ref(float x)
{
    const float e = (float)erf((double)x / 1.4142135623730951);
    return 0.5f * x * (1.0f + e);
}

__device__ __forceinline__ float act(float x) { return kExact ? gelu_ref(x) : gelu(x); }

// Block-wide reductions (fixed order: butterfly within the wave, then waves 0..3).
template <typename T>
__device__ __forceinline__ T block_max(T v, T *red)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const T u = __shfl_xor(v, o);
        v = u > v ? u : v;
    }
    const int wave = threadIdx.x / kWave;
    if (threadIdx.x % kWave == 0) red[wave] = v;
    __syncthreads();
    T r = red[0];
#pragma unroll
    for (int k = 1; k < kLearnWaves; ++k) r = red[k] > r ? red[k] : r;
    __syncthreads();
    return r;
}

template <typename T>
__device__ __forceinline__ T block_sum(T v, T *red)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int wave = threadIdx.x / kWave;
    if (threadIdx.x % kWave == 0) red[wave] = v;
    __syncthreads();
    T r = red[0];
#pragma unroll
    for (int k = 1; k < kLearnWaves; ++k) r += red[k];
    __syncthreads();
    return r;
}

// (key, index) maximum; equal keys go to the smaller index
template <typename T>
__device__ __forceinline__ int block_argmax(T key, int idx, T *rkey, int *ridx)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const T k2 = __shfl_xor(key, o);
        const int i2 = __shfl_xor(idx, o);
        if (k2 > key || (k2 == key && i2 < idx)) { key = k2; idx = i2; }
    }
    const int wave = threadIdx.x / kWave;
    if (threadIdx.x % kWave == 0) {
        rkey[wave] = key;
        ridx[wave] = idx;
    }
    __syncthreads();
    T bk = rkey[0];
    int bi = ridx[0];
#pragma unroll
    for (int k = 1; k < kLearnWaves; ++k) {
        const T k2 = rkey[k];
        const int i2 = ridx[k];
        if (k2 > bk || (k2 == bk && i2 < bi)) { bk = k2; bi = i2; }
    }
    __syncthreads();
    return bi;
}

__device__ __forceinline__ float lo_bf(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float hi_bf(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

__device__ __forceinline__ bf16x4 lo4(const uint4 &q)
{
    bf16x4 r;
    r[0] = (short)(q.x & 0xFFFFu); r[1] = (short)(q.x >> 16); r[2] = (short)(q.y & 0xFFFFu); r[3] = (short)(q.y >> 16);
    return r;
}

__device__ __forceinline__ bf16x4 hi4(const uint4 &q)
{
    bf16x4 r;
    r[0] = (short)(q.z & 0xFFFFu); r[1] = (short)(q.z >> 16); r[2] = (short)(q.w & 0xFFFFu); r[3] = (short)(q.w >> 16);
    return r;
}

// A fragment: the activation vector h (bfloat16, LDS) as every row, k = 16 kk + 4 (lane/16) + 0..3
__device__ __forceinline__ bf16x4 afrag(const bf16 *h, int kk, int lane)
{
    const uint2 u = *reinterpret_cast<const uint2 *>(h + 16 * kk + 4 * (lane >> 4));
    bf16x4 r;
    r[0] = (short)(u.x & 0xFFFFu); r[1] = (short)(u.x >> 16); r[2] = (short)(u.y & 0xFFFFu); r[3] = (short)(u.y >> 16);
    return r;
}

// Hidden layer on MFMA (tiled weights): out[n] = bf16(gelu(b[n] + sum_k W[n][k] in[k]));
// wave w takes output tiles 2w and 2w+1.
__device__ __forceinline__ void hidden_mfma(const uint16_t *wp, const float *bias, const bf16 *in, bf16 *out, int wave,
                                            int lane)
{
    bf16x4 a[8];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) a[kk] = afrag(in, kk, lane);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int tile = 2 * wave + q;
        const uint4 *bp = reinterpret_cast<const uint4 *>(wp) + (size_t)tile * 4 * kWave + lane;
        uint4 bq[4];
#pragma unroll
        for (int kp = 0; kp < 4; ++kp) bq[kp] = bp[kp * kWave];
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kp = 0; kp < 4; ++kp) {
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[2 * kp], lo4(bq[kp]), acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[2 * kp + 1], hi4(bq[kp]), acc, 0, 0, 0);
        }
        if (lane < 16) {
            const int n = 16 * tile + lane;
            out[n] = f2bf(act(acc[0] + bias[n]));
        }
    }
}

// Hidden layer with k-major weights, one output per thread, sequential FP32 sum in
// ascending k.
__device__ __forceinline__ void hidden_seq(const uint16_t *wt, const float *bias, const bf16 *in, bf16 *out, int tid)
{
    if (tid < kNetH) {
        float s = 0.f;
#pragma unroll 8
        for (int k = 0; k < kNetH; ++k) s += bf2f(wt[k * kNetH + tid]) * bf2f(in[k]);
        out[tid] = f2bf(act(s + bias[tid]));
    }
}

struct NetLds {
    const float *b1, *b2, *b3, *b4;   // biases (LDS copies)
    const uint32_t *occ;
    uint32_t *list;
    float *part;
    bf16 *h1, *h2, *h3;
    float *logit;
    double *redd;      // [kLearnWaves] doubles
    float *redf;       // [kLearnWaves] floats
    int *redi;         // [kLearnWaves] ints (scan totals, argmax indices)
    double *norm;      // FP32 build: ln of the FP64 sum of the weights of the current logits
    float *mxf;        // FP32 build: the largest of the current logits
};

// Block-wide scan of one FP64 value per thread in thread order: wave scans, then the
// wave totals added in order.  lo/hi = the sums before and through this thread (so
// the intervals [lo, hi) of consecutive threads meet exactly and cover [0, total));
// returns the total.  Both the normaliser and the voxel draw of the FP32 build use
// it, so they see the same total bit for bit.
__device__ __forceinline__ double block_scan(double v, double *red, int wave, int lane, double &lo, double &hi)
{
    double x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const double y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    double prev = __shfl_up(x, 1);
    if (lane == 0) prev = 0.0;
    __syncthreads();                  // earlier readers of red are done
    if (lane == kWave - 1) red[wave] = x;
    __syncthreads();
    double base = 0.0, total = 0.0;
#pragma unroll
    for (int q = 0; q < kLearnWaves; ++q) {
        if (q == wave) base = total;
        total += red[q];
    }
    lo = base + prev;
    hi = base + x;
    __syncthreads();
    return total;
}

// FP32 build: the categorical of the current logits is P(v) = w_v / sum_u w_u with
// w_v = expf(logit_v - max) in FP32 and the sum in FP64 in the order of block_scan
// (thread t owns voxels t + 256 j, summed over j in order).  The voxel draw realises
// exactly these weights, and the acceptance uses ln P(v) = ln w_v - ln sum, so the
// proposal density in the acceptance is the one the draw follows up to FP64 rounding.
__device__ __forceinline__ double weight_total(const NetLds &S, float mx, int tid, int wave, int lane)
{
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < kNetNV / kLT; ++j) v += (double)expf(S.logit[tid + kLT * j] - mx);
    double lo, hi;
    return block_scan(v, S.redd, wave, lane, lo, hi);
}

// ln P(v) of the current logits (lse: the value net_forward returned for them).
__device__ __forceinline__ double log_prob(const NetLds &S, double lse, int v)
{
    if (kExact) return (double)S.logit[v] - lse;
    return log((double)expf(S.logit[v] - S.mxf[0])) - S.norm[0];
}

// The network's logits for the occupancy without one particle in voxel `ex`
// (-1: none) into S.logit; returns the log-normaliser.  Block-wide.
__device__ double net_forward(const NetDev &net, const NetLds &S, int ex, int tid, int wave, int lane)
{
    // ascending list of occupied voxels, entries voxel | count << 16
    uint32_t cnt[16];
    int c = 0;
    {
        const uint4 *o4 = reinterpret_cast<const uint4 *>(S.occ + 16 * tid);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint4 u = o4[q];
            cnt[4 * q] = u.x; cnt[4 * q + 1] = u.y; cnt[4 * q + 2] = u.z; cnt[4 * q + 3] = u.w;
        }
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            cnt[j] -= (16 * tid + j == ex) ? 1u : 0u;
            c += cnt[j] != 0u;
        }
    }
    int incl = c;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int y = __shfl_up(incl, d);
        if (lane >= d) incl += y;
    }
    if (lane == kWave - 1) S.redi[wave] = incl;
    __syncthreads();
    int base = 0, m = 0;
#pragma unroll
    for (int k = 0; k < kLearnWaves; ++k) {
        const int t = S.redi[k];
        base += k < wave ? t : 0;
        m += t;
    }
    int pos = base + incl - c;
#pragma unroll
    for (int j = 0; j < 16; ++j)
        if (cnt[j]) S.list[pos++] = (uint32_t)(16 * tid + j) | (cnt[j] << 16);
    __syncthreads();

    // layer 1: b1 + sum over the list of count x W1 row
    // (entries are taken 8 at a time, their weight rows loaded before they are summed)
    if (kExact) {
        if (tid < kNetH) {
            float s = S.b1[tid];
            for (int j0 = 0; j0 < m; j0 += 8) {
                uint32_t e[8];
                bf16 wv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    e[u] = j0 + u < m ? S.list[j0 + u] : 0u;
                    wv[u] = net.w1[(size_t)(e[u] & 0xFFFFu) * kNetH + tid];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (j0 + u < m) s += (float)(e[u] >> 16) * bf2f(wv[u]);
            }
            S.h1[tid] = f2bf(act(s));
        }
    } else {
        // wave w takes entries w, w+4, ...; the four partial sums meet in LDS
        float a0 = 0.f, a1 = 0.f;
        const uint32_t *w1 = reinterpret_cast<const uint32_t *>(net.w1);
        for (int j0 = wave; j0 < m; j0 += 8 * kLearnWaves) {
            uint32_t e[8], wv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int j = j0 + u * kLearnWaves;
                e[u] = j < m ? S.list[j] : 0u;
                wv[u] = w1[(size_t)(e[u] & 0xFFFFu) * (kNetH / 2) + lane];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const float k = (float)(e[u] >> 16);     // 0 for the padding entries
                a0 += k * lo_bf(wv[u]);
                a1 += k * hi_bf(wv[u]);
            }
        }
        S.part[wave * kNetH + 2 * lane] = a0;
        S.part[wave * kNetH + 2 * lane + 1] = a1;
        __syncthreads();
        if (tid < kNetH) {
            float s = S.b1[tid];
#pragma unroll
            for (int k = 0; k < kLearnWaves; ++k) s += S.part[k * kNetH + tid];
            S.h1[tid] = f2bf(act(s));
        }
    }
    __syncthreads();
    if (kExact) hidden_seq(net.w2, S.b2, S.h1, S.h2, tid);
    else hidden_mfma(net.w2, S.b2, S.h1, S.h2, wave, lane);
    __syncthreads();
    if (kExact) hidden_seq(net.w3, S.b3, S.h2, S.h3, tid);
    else hidden_mfma(net.w3, S.b3, S.h2, S.h3, wave, lane);
    __syncthreads();

    if (kExact) {
        // output layer, thread t: voxels 16t .. 16t+15, sequential sums in ascending k;
        // the weights of 8 consecutive k are loaded before they are used
        float acc[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) acc[j] = 0.f;
        const uint4 *w4 = reinterpret_cast<const uint4 *>(net.w4) + 2 * tid;
        for (int k0 = 0; k0 < kNetH; k0 += 8) {
            uint4 q[8][2];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                q[u][0] = w4[(size_t)(k0 + u) * (kNetNV / 8)];
                q[u][1] = w4[(size_t)(k0 + u) * (kNetNV / 8) + 1];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const float hk = bf2f(S.h3[k0 + u]);
                const uint32_t wv[8] = {q[u][0].x, q[u][0].y, q[u][0].z, q[u][0].w,
                                        q[u][1].x, q[u][1].y, q[u][1].z, q[u][1].w};
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    acc[2 * j] += lo_bf(wv[j]) * hk;
                    acc[2 * j + 1] += hi_bf(wv[j]) * hk;
                }
            }
        }
#pragma unroll
        for (int j = 0; j < 16; ++j) S.logit[16 * tid + j] = acc[j] + S.b4[16 * tid + j];
        __syncthreads();
        double mx = -INFINITY;
#pragma unroll
        for (int q = 0; q < kNetNV / kLT; ++q) {
            const double v = (double)S.logit[tid + kLT * q];
            mx = v > mx ? v : mx;
        }
        mx = block_max(mx, S.redd);
        double sum = 0.0;
#pragma unroll
        for (int q = 0; q < kNetNV / kLT; ++q) sum += exp((double)S.logit[tid + kLT * q] - mx);
        sum = block_sum(sum, S.redd);
        return mx + log(sum);
    } else {
        // output layer on MFMA: wave w takes tiles 64w .. 64w+63 (16 voxels each), in
        // stages of 4 tiles; the next stage's weights are in flight while a stage computes
        bf16x4 a[8];
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) a[kk] = afrag(S.h3, kk, lane);
        constexpr int TS = 4;
        const uint4 *wp = reinterpret_cast<const uint4 *>(net.w4) + (size_t)(64 * wave) * 4 * kWave + lane;
        auto load = [&](uint4 (&b)[TS][4], int t) {
#pragma unroll
            for (int u = 0; u < TS; ++u)
#pragma unroll
                for (int kp = 0; kp < 4; ++kp) b[u][kp] = wp[((size_t)(t + u) * 4 + kp) * kWave];
        };
        auto compute = [&](const uint4 (&b)[TS][4], int t) {
#pragma unroll
            for (int u = 0; u < TS; ++u) {
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kp = 0; kp < 4; ++kp) {
                    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[2 * kp], lo4(b[u][kp]), acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[2 * kp + 1], hi4(b[u][kp]), acc, 0, 0, 0);
                }
                if (lane < 16) {
                    const int v = 16 * (64 * wave + t + u) + lane;
                    S.logit[v] = acc[0] + S.b4[v];
                }
            }
        };
        uint4 bA[TS][4], bB[TS][4];
        load(bA, 0);
        for (int t = 0; t < 64; t += 2 * TS) {
            load(bB, t + TS);
            compute(bA, t);
            if (t + 2 * TS < 64) load(bA, t + 2 * TS);
            compute(bB, t + TS);
        }
        __syncthreads();
        float mx = -INFINITY;
#pragma unroll
        for (int q = 0; q < kNetNV / kLT; ++q) mx = fmaxf(mx, S.logit[tid + kLT * q]);
        mx = block_max(mx, S.redf);
        const double lsum = log(weight_total(S, mx, tid, wave, lane));
        if (tid == 0) {
            S.norm[0] = lsum;
            S.mxf[0] = mx;
        }
        __syncthreads();
        return (double)mx + lsum;
    }
}

// Voxel draw from softmax(logit) (block-wide).
// FP64 build (the oracle's draw): Gumbel-max, argmax_v logit_v - ln(-ln u_v); thread
// t takes the Philox blocks 16 + t + 256 r, r = 0..3, i.e. voxels 4 (t + 256 r) .. +3.
// FP32 build: inverse CDF with one 53-bit uniform u (words x, y of Philox block 16).
// Thread t owns voxels t + 256 j, j = 0..15, with the FP32 weights w_v of log_prob; the
// FP64 scan of the threads' sums cuts [0, total) into contiguous intervals [lo_t, hi_t),
// and the thread whose interval holds u total (< total, as u <= 1 - 2^-53) walks its
// weights in FP64.  Each voxel is drawn with probability w_v / total up to the FP64
// rounding of the running sums (a few 2^-53 of the total per voxel).
__device__ int draw_voxel(const NetLds &S, double lse, uint32_t t, uint32_t sweep, uint32_t w, uint32_t k0,
                          uint32_t k1, int tid)
{
    if (kExact) {
        double best = -INFINITY;
        int arg = 0x7fffffff;
#pragma unroll
        for (int r = 0; r < kNetNV / (4 * kLT); ++r) {
            const int b = tid + kLT * r;
            const uint4 R = philox4x32_10(make_uint4(t, sweep, w, 16u + (uint32_t)b), k0, k1);
            const uint32_t words[4] = {R.x, R.y, R.z, R.w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int v = 4 * b + q;
                const double key = (double)S.logit[v] - log(-log(uniform_open(words[q])));
                if (key > best || (key == best && v < arg)) { best = key; arg = v; }
            }
        }
        return block_argmax(best, arg, S.redd, S.redi);
    } else {
        constexpr int P = kNetNV / kLT;
        const int wave = tid / kWave, lane = tid % kWave;
        const float mx = S.mxf[0];
        float p[P];
        double v = 0.0;
#pragma unroll
        for (int j = 0; j < P; ++j) {
            p[j] = expf(S.logit[tid + kLT * j] - mx);
            v += (double)p[j];
        }
        double lo, hi;
        if (tid == 0) S.redi[0] = 0;
        const double total = block_scan(v, S.redd, wave, lane, lo, hi);
        const uint4 R = philox4x32_10(make_uint4(t, sweep, w, 16u), k0, k1);
        const double target = uniform53(R.x, R.y) * total;      // in [0, total)
        if (lo <= target && target < hi) {
            // the first voxel whose running FP64 sum passes the target; if rounding
            // leaves the walk short of hi, the last voxel of positive weight
            double c = lo;
            int pick = -1, last = 0;
#pragma unroll
            for (int j = 0; j < P; ++j) {
                if (p[j] > 0.f) last = j;
                c += (double)p[j];
                if (pick < 0 && target < c) pick = j;
            }
            S.redi[0] = tid + kLT * (pick >= 0 ? pick : last);
        }
        __syncthreads();
        const int vv = S.redi[0];
        __syncthreads();
        return vv;
    }
}

__global__ void __launch_bounds__(kLT) learned_kernel(SweepArgs a, LearnArgs l)
{
    extern __shared__ __align__(32) unsigned char smem[];
    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    const int w = l.block_walker[blockIdx.x];
    const int cid = l.walker_class[w];
    const ClassDev &C = a.cls[cid];
    const NetDev &net = l.net[cid];
    const double alpha = l.alpha[cid];
    const LearnLds L = learn_lds(a.max_slab_len, a.gas_stride, (int)sizeof(Real));
    Real4 *slab = reinterpret_cast<Real4 *>(smem + L.slab);
    double *lnk = reinterpret_cast<double *>(smem + L.lnk);
    double *xch = reinterpret_cast<double *>(smem + L.xch);          // [parity][wave][value, core]
    Real4 *gas = reinterpret_cast<Real4 *>(smem + L.gas);
    int *vox = reinterpret_cast<int *>(smem + L.vox);
    uint32_t *occ = reinterpret_cast<uint32_t *>(smem + L.occ);
    NetLds S;
    S.occ = occ;
    S.list = reinterpret_cast<uint32_t *>(smem + L.list);
    S.part = reinterpret_cast<float *>(smem + L.part);
    S.h1 = reinterpret_cast<bf16 *>(smem + L.hid);
    S.h2 = S.h1 + kNetH;
    S.h3 = S.h2 + kNetH;
    S.logit = reinterpret_cast<float *>(smem + L.logit);
    {
        float *bias = reinterpret_cast<float *>(smem + L.bias);
        if (alpha > 0.0) {
            for (int k = tid; k < kNetNV; k += kLT) bias[k] = net.b4[k];
            for (int k = tid; k < 3 * kNetH; k += kLT)
                bias[kNetNV + k] = k < kNetH ? net.b1[k] : (k < 2 * kNetH ? net.b2[k - kNetH] : net.b3[k - 2 * kNetH]);
        }
        S.b4 = bias;
        S.b1 = bias + kNetNV;
        S.b2 = S.b1 + kNetH;
        S.b3 = S.b2 + kNetH;
    }
    S.redd = reinterpret_cast<double *>(smem + L.red);
    S.redf = reinterpret_cast<float *>(S.redd + kLearnWaves);
    S.redi = reinterpret_cast<int *>(S.redf + kLearnWaves);
    S.norm = reinterpret_cast<double *>(S.redi + kLearnWaves);
    S.mxf = reinterpret_cast<float *>(S.norm + 1);

    const int slab_len = C.slab_len;
    for (int k = tid; k < slab_len; k += kLT) {
#if defined(REGC_FP64)
        const double *src = a.slab4 + 4 * (size_t)(C.slab_off + k);
#else
        const float *src = a.slab4f + 4 * (size_t)(C.slab_off + k);
#endif
        Real4 v;
        v.x = src[0]; v.y = src[1]; v.z = src[2]; v.w = 0;
        slab[k] = v;
    }
    for (int k = tid; k < a.gas_stride + 2; k += kLT) lnk[k] = a.lnk[k];
    for (int k = tid; k < kNetNV; k += kLT) occ[k] = 0u;

    Grid g;
    g.gx = (double)kNetGrid / C.lx;
    g.gy = (double)kNetGrid / C.ly;
    g.gz = (double)kNetGrid / (C.zhi - C.zlo);
    g.zlo = C.zlo;
    g.cx = C.lx / (double)kNetGrid;
    g.cy = C.ly / (double)kNetGrid;
    g.cz = (C.zhi - C.zlo) / (double)kNetGrid;

    const int n_max = C.n_max;
    const int K = C.trials;
    int n = a.n[w];
    double e = a.e[w];
    const int label = a.label[w];
    const int sg = C.state_off + label;
    const double beta = a.beta[sg];
    const double lnz = a.lnz[sg];
    const double lnzv = lnz + C.lnv;
    __syncthreads();
    {
        const double *src = a.xyz + (size_t)w * a.xyz_stride * 3;
        for (int k = tid; k < n; k += kLT) {
            Real4 v;
            v.x = (Real)src[3 * k]; v.y = (Real)src[3 * k + 1]; v.z = (Real)src[3 * k + 2]; v.w = 0;
            gas[k] = v;
            const int vv = voxel_of(g, (double)v.x, (double)v.y, (double)v.z);
            vox[k] = vv;
            atomicAdd(occ + vv, 1u);
        }
    }
    __syncthreads();

    Box b;
    b.lx = (Real)C.lx; b.ly = (Real)C.ly; b.hx = (Real)C.half_lx; b.hy = (Real)C.half_ly;
    b.ix = (Real)C.inv_lx; b.iy = (Real)C.inv_ly;
    Pair gg, gs;
    gg.sig2 = (Real)a.pot.sig2_gg; gg.eps4 = (Real)a.pot.eps4_gg; gg.shift = (Real)a.pot.shift_gg;
    gg.rc2 = (Real)a.pot.rc2; gg.hc2 = (Real)a.pot.hc2_gg;
    gs.sig2 = (Real)a.pot.sig2_gs; gs.eps4 = (Real)a.pot.eps4_gs; gs.shift = (Real)a.pot.shift_gs;
    gs.rc2 = gg.rc2; gs.hc2 = (Real)a.pot.hc2_gs;
    const bool ideal = a.pot.ideal != 0;
    SlabView sv;
    sv.atoms = slab; sv.len = slab_len; sv.bins = C.bins;
    sv.ncx = C.ncx; sv.ncy = C.ncy; sv.cap = C.cap;
    sv.inv_cap = C.bins ? 1.0f / (float)C.cap : 0.f;
    sv.inv_cw_x = (Real)C.inv_cw_x; sv.inv_cw_y = (Real)C.inv_cw_y;
    sv.top_plus_rc = (Real)(C.slab_top + sqrt(a.pot.rc2));
    const double lx = C.lx, ly = C.ly, zlo = C.zlo, zhi = C.zhi, H = C.zhi - C.zlo;
    const double md = a.max_disp;
    const double tinv = 1.0 / beta;

    uint32_t stat = 0;          // wave 0: lane k < kNStat holds counter k
    uint32_t useful = 0;        // (unused pair counter of the shared helper)
    uint32_t xcount = 0;        // energy exchanges so far: consecutive ones use alternate slots
    bool cached = false;        // S.logit / lse hold the network output of the current occupancy
    double lse = 0.0;
    unsigned long long ev_pass = 0, ev_hit = 0, ev_net = 0, ev_netacc = 0;

    const int64_t sweep_first = a.clock ? a.clock[0] + a.sweep0 : a.sweep0;
    for (int it = 0; it < a.n_sweeps; ++it) {
        const int64_t sweep = sweep_first + it;
        const bool tracing = a.trace_bits != nullptr && (sweep - a.trace_sweep0) < a.trace_cap &&
                             sweep >= a.trace_sweep0;
        for (int t0 = 0; t0 < K; t0 += 32) {
            const uint4 R = philox4x32_10(
                make_uint4((uint32_t)(t0 + (lane >> 1)), (uint32_t)sweep, (uint32_t)w, (uint32_t)(lane & 1)),
                a.key0, a.key1);
            const double f0 = uniform_open(R.z), f1 = uniform_open(R.w), f2 = uniform_open(R.x);
            const double f3 = log(uniform53(R.y, R.z));
            const double fm = uniform_open(R.w);           // B lanes: the mixture uniform (B3)
            const int tn = K - t0 < 32 ? K - t0 : 32;
            uint32_t bits = 0;
            for (int tt = 0; tt < tn; ++tt) {
                const uint32_t A0 = bcast(R.x, 2 * tt), A1 = bcast(R.y, 2 * tt);
                const int kind = (uint64_t)A0 < a.th_disp ? 0 : ((uint64_t)A0 < a.th_ins ? 1 : 2);
                if (wave == 0) stat += lane == 2 * kind;
                bool accepted = false;
                if (kind == 1 ? n >= n_max : n == 0) {
                    if (wave == 0) stat += lane == (kind == 1 ? 6 : 7);
                } else {
                    const double lnU = bcast(f3, 2 * tt + 1);
                    const double ux = bcast(f0, 2 * tt), uy = bcast(f1, 2 * tt), uz = bcast(f2, 2 * tt + 1);
                    const int i = kind == 1 ? -1 : (int)(((uint64_t)A1 * (uint64_t)n) >> 32);
                    const Real4 o = gas[kind == 1 ? 0 : i];
                    const int vold = kind == 1 ? -1 : vox[i];
                    double px = 0.0, py = 0.0, pz = 0.0, c = 0.0;
                    bool wall = false;
                    if (kind == 0) {
                        px = (double)o.x + md * (2.0 * ux - 1.0);
                        py = (double)o.y + md * (2.0 * uy - 1.0);
                        pz = (double)o.z + md * (2.0 * uz - 1.0);
                        if (px < 0.0) px += lx; else if (px >= lx) px -= lx;
                        if (py < 0.0) py += ly; else if (py >= ly) py -= ly;
                        wall = pz < zlo || pz > zhi;
                    } else if (alpha == 0.0) {
                        // a class without a network: the plain method (q = 1/V)
                        if (kind == 1) {
                            px = lx * ux;
                            py = ly * uy;
                            pz = zlo + H * uz;
                        }
                        c = kind == 1 ? lnzv - lnk[n + 1] : lnk[n] - lnzv;
                    } else {
                        // network output for occ(X) (insertion, cached while X's occupancy
                        // stands) or occ(X \ i) (removal)
                        if (kind == 2 || !cached) {
                            lse = net_forward(net, S, kind == 2 ? vold : -1, tid, wave, lane);
                            ++ev_pass;
                        } else {
                            ++ev_hit;
                        }
                        cached = kind == 1;
                        int v;
                        if (kind == 1) {
                            if (bcast(fm, 2 * tt + 1) < alpha) {
                                v = draw_voxel(S, lse, (uint32_t)(t0 + tt), (uint32_t)sweep, (uint32_t)w, a.key0,
                                               a.key1, tid);
                                px = ((double)(v & (kNetGrid - 1)) + ux) * g.cx;
                                py = ((double)((v >> 4) & (kNetGrid - 1)) + uy) * g.cy;
                                pz = zlo + ((double)(v >> 8) + uz) * g.cz;
                                // a point rounded onto a neighbouring voxel is not a draw of v
                                wall = voxel_of(g, (double)(Real)px, (double)(Real)py, (double)(Real)pz) != v;
                                ++ev_net;
                            } else {
                                px = lx * ux;
                                py = ly * uy;
                                pz = zlo + H * uz;
                                v = voxel_of(g, (double)(Real)px, (double)(Real)py, (double)(Real)pz);
                            }
                        } else {
                            v = vold;
                        }
                        const double lnp = log_prob(S, lse, v);
                        const double lq = log1p(alpha * (exp(lnp) * (double)kNetNV - 1.0));
                        c = kind == 1 ? (lnzv - lnk[n + 1]) - lq : (lnk[n] - lnzv) + lq;
                    }
                    if (wall) {
                        if (wave == 0) stat += lane == 8;
                    } else {
                        const double thr = (c - lnU) * tinv;
                        const Real qx = (Real)px, qy = (Real)py, qz = (Real)pz;
                        double de = 0.0;
                        bool core = false;
                        if (!ideal) {
                            Real pd;
                            if (kind == 0)
                                pd = partial_delta<true, true, kLearnWaves, false>(gas, n, i, sv, b, gg, gs, lane, wave,
                                                                                   qx, qy, qz, o.x, o.y, o.z, nullptr,
                                                                                   nullptr, core, useful);
                            else if (kind == 1)
                                pd = partial_delta<true, false, kLearnWaves, false>(gas, n, -1, sv, b, gg, gs, lane,
                                                                                    wave, qx, qy, qz, qx, qy, qz,
                                                                                    nullptr, nullptr, core, useful);
                            else
                                pd = partial_delta<false, true, kLearnWaves, false>(gas, n, i, sv, b, gg, gs, lane,
                                                                                    wave, o.x, o.y, o.z, o.x, o.y, o.z,
                                                                                    nullptr, nullptr, core, useful);
                            double *mine = xch + ((xcount & 1) * kLearnWaves + wave) * 2;
                            if (lane == 0) {
                                mine[0] = (double)pd;
                                mine[1] = core ? 1.0 : 0.0;
                            }
                            __syncthreads();
                            const double *x0 = xch + (xcount & 1) * kLearnWaves * 2;
                            de = x0[0];
                            double cf = x0[1];
#pragma unroll
                            for (int k = 1; k < kLearnWaves; ++k) {
                                de += x0[2 * k];
                                cf += x0[2 * k + 1];
                            }
                            core = cf != 0.0;
                            ++xcount;
                        }
                        if (core && kind != 2) {
                            if (wave == 0) stat += lane == 9;
                        } else if (de <= thr) {
                            accepted = true;
                            if (wave == 0) stat += lane == 2 * kind + 1;
                            e += de;
                            const int vnew = kind == 2 ? -1 : voxel_of(g, (double)qx, (double)qy, (double)qz);
                            __syncthreads();       // every wave has read gas[] and vox[] of this trial
                            if (tid == 0) {
                                Real4 nv; nv.x = qx; nv.y = qy; nv.z = qz; nv.w = 0;
                                if (kind == 0) {
                                    gas[i] = nv;
                                    if (vnew != vold) {
                                        occ[vold] -= 1u;
                                        occ[vnew] += 1u;
                                        vox[i] = vnew;
                                    }
                                } else if (kind == 1) {
                                    gas[n] = nv;
                                    vox[n] = vnew;
                                    occ[vnew] += 1u;
                                } else {
                                    occ[vold] -= 1u;
                                    if (i != n - 1) {
                                        gas[i] = gas[n - 1];
                                        vox[i] = vox[n - 1];
                                    }
                                }
                            }
                            if (kind == 0) {
                                if (vnew != vold) cached = false;
                            } else if (kind == 1) {
                                n += 1;
                                cached = false;
                                if (bcast(fm, 2 * tt + 1) < alpha) ++ev_netacc;
                            } else {
                                n -= 1;
                                cached = true;     // the last pass was on occ(X \ i), the new X
                            }
                        }
                    }
                }
                if (accepted) {
                    bits |= 1u << tt;
                    __syncthreads();
                }
            }
            if (tracing && tid == 0)
                a.trace_bits[((size_t)(sweep - a.trace_sweep0) * a.n_walkers + w) * a.trace_words + (t0 >> 5)] = bits;
        }
        if (tid == 0) {
            if (tracing) a.trace_n[(size_t)(sweep - a.trace_sweep0) * a.n_walkers + w] = n;
            if (a.sample_every > 0 && (sweep + 1) % a.sample_every == 0) {
                const int64_t rec = (sweep + 1) / a.sample_every - 1 - a.rec_base;
                const size_t idx = (size_t)rec * a.n_walkers + w;
                a.samp_e[idx] = e;
                a.samp_n[idx] = n;
                a.samp_s[idx] = label;
                atomicAdd(a.hist + (size_t)sg * a.hist_stride + n, 1ull);
            }
        }
    }

    __syncthreads();
    {
        double *dst = a.xyz + (size_t)w * a.xyz_stride * 3;
        for (int k = tid; k < n; k += kLT) {
            const Real4 v = gas[k];
            dst[3 * k] = (double)v.x; dst[3 * k + 1] = (double)v.y; dst[3 * k + 2] = (double)v.z;
        }
    }
    if (wave == 0 && lane < kNStat && stat) atomicAdd(a.stats + (size_t)sg * kNStat + lane, (unsigned long long)stat);
    if (tid == 0) {
        a.n[w] = n;
        a.e[w] = e;
        if (l.evals) {
            atomicAdd(l.evals + 0, ev_pass);
            atomicAdd(l.evals + 1, ev_hit);
            atomicAdd(l.evals + 2, ev_net);
            atomicAdd(l.evals + 3, ev_netacc);
        }
    }
}

// The sampler's network on given configurations (one workgroup each): the occupancy
// of the particles (positions rounded to Real, as the sampler holds them) without
// particle skip[c] (-1: none), then net_forward.  logits [c][4096], lse [c] (the
// normaliser the sampler returns), lnp [c][4096] = ln P(v) as the acceptance uses it.
__global__ void __launch_bounds__(kLT) net_eval_kernel(NetDev net, const ClassDev *cls, int cid, int stride,
                                                       const double *xyz, const int32_t *n_conf,
                                                       const int32_t *skip, float *logits, double *lse_out,
                                                       double *lnp_out)
{
    extern __shared__ __align__(32) unsigned char smem[];
    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    const int c = blockIdx.x;
    const ClassDev &C = cls[cid];
    const LearnLds L = learn_lds(0, stride, (int)sizeof(Real));
    uint32_t *occ = reinterpret_cast<uint32_t *>(smem + L.occ);
    int *vox = reinterpret_cast<int *>(smem + L.vox);
    NetLds S;
    S.occ = occ;
    S.list = reinterpret_cast<uint32_t *>(smem + L.list);
    S.part = reinterpret_cast<float *>(smem + L.part);
    S.h1 = reinterpret_cast<bf16 *>(smem + L.hid);
    S.h2 = S.h1 + kNetH;
    S.h3 = S.h2 + kNetH;
    S.logit = reinterpret_cast<float *>(smem + L.logit);
    float *bias = reinterpret_cast<float *>(smem + L.bias);
    for (int k = tid; k < kNetNV; k += kLT) bias[k] = net.b4[k];
    for (int k = tid; k < 3 * kNetH; k += kLT)
        bias[kNetNV + k] = k < kNetH ? net.b1[k] : (k < 2 * kNetH ? net.b2[k - kNetH] : net.b3[k - 2 * kNetH]);
    S.b4 = bias;
    S.b1 = bias + kNetNV;
    S.b2 = S.b1 + kNetH;
    S.b3 = S.b2 + kNetH;
    S.redd = reinterpret_cast<double *>(smem + L.red);
    S.redf = reinterpret_cast<float *>(S.redd + kLearnWaves);
    S.redi = reinterpret_cast<int *>(S.redf + kLearnWaves);
    S.norm = reinterpret_cast<double *>(S.redi + kLearnWaves);
    S.mxf = reinterpret_cast<float *>(S.norm + 1);
    for (int k = tid; k < kNetNV; k += kLT) occ[k] = 0u;
    Grid g;
    g.gx = (double)kNetGrid / C.lx;
    g.gy = (double)kNetGrid / C.ly;
    g.gz = (double)kNetGrid / (C.zhi - C.zlo);
    g.zlo = C.zlo;
    __syncthreads();
    const int n = n_conf[c];
    const double *x = xyz + (size_t)c * stride * 3;
    for (int k = tid; k < n; k += kLT) {
        const int vv = voxel_of(g, (double)(Real)x[3 * k], (double)(Real)x[3 * k + 1], (double)(Real)x[3 * k + 2]);
        vox[k] = vv;
        atomicAdd(occ + vv, 1u);
    }
    __syncthreads();
    const int ex = skip[c] >= 0 && skip[c] < n ? vox[skip[c]] : -1;
    const double lse = net_forward(net, S, ex, tid, wave, lane);
    for (int v = tid; v < kNetNV; v += kLT) {
        logits[(size_t)c * kNetNV + v] = S.logit[v];
        lnp_out[(size_t)c * kNetNV + v] = log_prob(S, lse, v);
    }
    if (tid == 0) lse_out[c] = lse;
}

}  // namespace fp64 / fp32

using namespace REGC_PREC;

hipError_t LEARNED_LAUNCH(const SweepArgs &a, const LearnArgs &l, size_t smem, hipStream_t s)
{
    hipLaunchKernelGGL(learned_kernel, dim3(a.n_walkers), dim3(kLT), smem, s, a, l);
    return hipGetLastError();
}

hipError_t NET_EVAL_LAUNCH(const NetDev &net, const ClassDev *cls, int cid, int stride, int n_conf, const double *xyz,
                           const int32_t *n, const int32_t *skip, float *logits, double *lse, double *lnp,
                           hipStream_t s)
{
    const size_t smem = learn_lds(0, stride, (int)sizeof(Real)).total;
    hipLaunchKernelGGL(net_eval_kernel, dim3(n_conf), dim3(kLT), smem, s, net, cls, cid, stride, xyz, n, skip, logits,
                       lse, lnp);
    return hipGetLastError();
}

}  // namespace regc
