// mlp.hip -- the learned insertion proposal network on the GPU: forward, backward,
// Adam and the training loop, bfloat16 operands on MFMA with FP32 accumulation.
//
// Network (an extension of the REGC method, not in the paper): the 16^3 occupancy
// grid of a configuration -> 128 -> 128 -> 128 -> 4096 logits over insertion
// voxels; GELU (erf form) after each hidden layer.  Layer 1 is a gather: the
// occupancy has at most n_max non-zero voxels, so its product with W1 is the sum
// of the W1 columns of the occupied voxels (one per particle, in particle order).
// Layers 2-4 and the weight/activation gradients are MFMA GEMMs
// (v_mfma_f32_16x16x16_bf16: lane l holds A row l%16 and B column l%16 at
// k = 4*(l/16)..+3; the result element D[4*(l/16)+r][l%16] sits in register r).
// Rounding points: weights and hidden activations are rounded to bfloat16
// (nearest even) before each product; pre-activations, logits, softmax, the
// gradient sums and the Adam state are FP32.
//
// Training example: a stored configuration, one particle i of it; input = the
// occupancy without i, target = the voxel of i; loss = cross-entropy.
// Parameter vector layout (FP32, also the ABI's): W1 [4096][128] (voxel-major),
// b1 [128], W2 [128][128] ([out][in]), b2, W3, b3, W4 [4096][128] ([voxel][in]), b4 [4096].
#include <algorithm>
#include <cmath>
#include <vector>

#include "host_util.h"
#include "mlp_dev.h"
#include "philox_dev.h"
#include "learn_dev.h"

namespace regc {
namespace mlpk {

constexpr int NV = 4096, H = 128;
constexpr int kSplitK = 16;   // K = 4096 products split 16 ways
constexpr size_t OFF_W1 = 0, OFF_B1 = OFF_W1 + (size_t)NV * H, OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + (size_t)H * H,
                 OFF_W3 = OFF_B2 + H, OFF_B3 = OFF_W3 + (size_t)H * H, OFF_W4 = OFF_B3 + H,
                 OFF_B4 = OFF_W4 + (size_t)NV * H, NPARAM = OFF_B4 + NV;

enum { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_GELU = 2 };

// C[M][N] = sum_k A(m,k) B(k,n); A(m,k) = TA ? A[k*lda+m] : A[m*lda+k],
// B(k,n) = TB ? B[n*ldb+k] : B[k*ldb+n].  Block tile 64x64 (4 waves of 32x32,
// 2x2 MFMA blocks each); M, N multiples of 64, K a multiple of 16 (host-checked).
// EPI_BIAS adds bias[n]; EPI_BIAS_GELU also writes act = bf16(gelu(C)).
template <bool TA, bool TB, int EPI>
__global__ void __launch_bounds__(256) gemm_bf16(int M, int N, int K, const bf16 *__restrict__ A, int lda,
                                              const bf16 *__restrict__ B, int ldb, float *__restrict__ C, int ldc,
                                              const float *__restrict__ bias, bf16 *__restrict__ act, int ldact)
{
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int m0 = blockIdx.y * 64 + (wave / 2) * 32;
    const int n0 = blockIdx.x * 64 + (wave % 2) * 32;
    const int lr = lane % 16, lk = 4 * (lane / 16);
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    // split K: block z takes k in [z K / Z, (z+1) K / Z) and writes the z-th of Z partial results
    const int kspan = K / (int)gridDim.z, kbeg = (int)blockIdx.z * kspan;
    C += (size_t)blockIdx.z * M * ldc;
    for (int k0 = kbeg; k0 < kbeg + kspan; k0 += 16) {
        bf16x4 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int m = m0 + 16 * i + lr;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = k0 + lk + q;
                a[i][q] = (short)(TA ? A[(size_t)k * lda + m] : A[(size_t)m * lda + k]);
            }
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + 16 * j + lr;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = k0 + lk + q;
                b[j][q] = (short)(TB ? B[(size_t)n * ldb + k] : B[(size_t)k * ldb + n]);
            }
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + 16 * i + 4 * (lane / 16) + r;
                const int n = n0 + 16 * j + lane % 16;
                float v = acc[i][j][r];
                if (EPI != EPI_STORE) v += bias[n];
                C[(size_t)m * ldc + n] = v;
                if (EPI == EPI_BIAS_GELU) act[(size_t)m * ldact + n] = f2bf(gelu(v));
            }
}

// out = sum over z of the Z partial results part[z] (count values each), z in order
__global__ void sum_partials(int Z, size_t count, const float *part, float *out)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    float s = part[i];
    for (int z = 1; z < Z; ++z) s += part[(size_t)z * count + i];
    out[i] = s;
}

// Layer 1: a1[b] = b1 + sum of W1 columns of the occupied voxels (particles j != excl[b]).
__global__ void __launch_bounds__(128) l1_forward(int nmax, const uint16_t *vox, const int32_t *n, const int32_t *excl,
                                              const bf16 *W1, const float *b1, float *a1, bf16 *h1)
{
    const int b = blockIdx.x, k = threadIdx.x;
    float acc = b1[k];
    const int nb = n[b], ex = excl[b];
    for (int j = 0; j < nb; ++j)
        if (j != ex) acc += bf2f(W1[(size_t)vox[(size_t)b * nmax + j] * H + k]);
    a1[(size_t)b * H + k] = acc;
    h1[(size_t)b * H + k] = f2bf(gelu(acc));
}

__device__ __forceinline__ float block_reduce(float v, float *sh, bool is_max)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const float t = __shfl_xor(v, o);
        v = is_max ? fmaxf(v, t) : v + t;
    }
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    float r = sh[0];
    for (int w = 1; w < (int)(blockDim.x / 64); ++w) r = is_max ? fmaxf(r, sh[w]) : r + sh[w];
    return r;
}

// Row-wise log-softmax cross-entropy: loss[b] = lse - logit[target]; the logit
// gradient d = (softmax - onehot) / B in FP32 and bfloat16.
__global__ void __launch_bounds__(256) softmax_xent(int B, const float *logits, const int32_t *target, float *loss,
                                                 float *d32, bf16 *d16)
{
    __shared__ float sh[8];
    const int b = blockIdx.x;
    const float *row = logits + (size_t)b * NV;
    float mx = -INFINITY;
    for (int v = threadIdx.x; v < NV; v += blockDim.x) mx = fmaxf(mx, row[v]);
    mx = block_reduce(mx, sh, true);
    float s = 0.f;
    for (int v = threadIdx.x; v < NV; v += blockDim.x) s += expf(row[v] - mx);
    s = block_reduce(s, sh, false);
    const float lse = mx + logf(s);
    const int t = target[b];          // < 0: no example in this slot (zero loss and gradient)
    if (threadIdx.x == 0) loss[b] = t >= 0 ? lse - row[t] : 0.0f;
    const float inv_b = t >= 0 ? 1.0f / (float)B : 0.0f;
    for (int v = threadIdx.x; v < NV; v += blockDim.x) {
        const float g = (expf(row[v] - lse) - (v == t ? 1.0f : 0.0f)) * inv_b;
        d32[(size_t)b * NV + v] = g;
        d16[(size_t)b * NV + v] = f2bf(g);
    }
}

__global__ void gelu_backward(int count, const float *dh, const float *a, float *da, bf16 *da16)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float v = dh[i] * gelu_grad(a[i]);
    da[i] = v;
    da16[i] = f2bf(v);
}

// out[n] = sum_m X[m][n]: a block of 256 threads takes 64 columns; thread (g, c)
// sums rows g, g+4, ... of column c in order, the four partial sums are added in
// the order g = 0..3 (deterministic).
__global__ void __launch_bounds__(256) colsum(int M, int N, const float *X, float *out)
{
    __shared__ float part[4][64];
    const int c = threadIdx.x % 64, g = threadIdx.x / 64;
    const int col = blockIdx.x * 64 + c;
    float s = 0.f;
    if (col < N)
        for (int m = g; m < M; m += 4) s += X[(size_t)m * N + col];
    part[g][c] = s;
    __syncthreads();
    if (g == 0 && col < N) out[col] = ((part[0][c] + part[1][c]) + part[2][c]) + part[3][c];
}

// dW1[voxel][k] += da1[b][k] for every occupied voxel of example b
__global__ void __launch_bounds__(128) l1_backward(int nmax, const uint16_t *vox, const int32_t *n, const int32_t *excl,
                                               const float *da1, float *gW1)
{
    const int b = blockIdx.x, k = threadIdx.x;
    const int nb = n[b], ex = excl[b];
    const float g = da1[(size_t)b * H + k];
    for (int j = 0; j < nb; ++j)
        if (j != ex) atomicAdd(gW1 + (size_t)vox[(size_t)b * nmax + j] * H + k, g);
}

// Adam with bias correction (Kingma & Ba, ICLR 2015); writes the bfloat16 copy.
__global__ void adam_update(size_t count, float *p, const float *g, float *m, float *v, float lr, float c1, float c2,
                            float beta1, float beta2, float eps, bf16 *p16)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = beta1 * m[i] + (1.f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    p16[i] = f2bf(pi);
}

__global__ void to_bf16(size_t count, const float *x, bf16 *y)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) y[i] = f2bf(x[i]);
}

// Training batch from a device data set of configurations (voxel lists): example
// e = (53-bit word) mod n_examples and left-out particle i = floor(U' * N_e) from
// Philox counter (slot, step, 0xFFFFFFFF, 5) with the given key.  Empty
// configurations are passed over for the next ones (at most 256); a slot left
// without particles gets target -1 (no loss, no gradient).
__global__ void make_batch(int B, int nmax, int64_t n_examples, const uint16_t *set_vox, const int32_t *set_n,
                           int64_t step, uint32_t k0, uint32_t k1, uint16_t *vox, int32_t *n, int32_t *excl,
                           int32_t *target)
{
    const int b = blockIdx.x;
    const uint4 r = philox4x32_10(make_uint4((uint32_t)b, (uint32_t)step, 0xFFFFFFFFu, 5u), k0, k1);
    uint64_t pick = (uint64_t)(((((uint64_t)r.x << 32) | r.y) >> 11) % (uint64_t)n_examples);
    int nb = set_n[pick];
    for (int tries = 0; nb == 0 && tries < 256; ++tries) {
        pick = pick + 1 == (uint64_t)n_examples ? 0 : pick + 1;
        nb = set_n[pick];
    }
    for (int j = threadIdx.x; j < nmax; j += blockDim.x)
        vox[(size_t)b * nmax + j] = j < nb ? set_vox[pick * nmax + j] : 0;
    if (threadIdx.x == 0) {
        const int i = nb > 0 ? (int)(((uint64_t)r.z * (uint64_t)nb) >> 32) : -1;
        n[b] = nb;
        excl[b] = i;
        target[b] = i >= 0 ? (int32_t)set_vox[pick * nmax + i] : -1;
    }
}

// Flags a training set with an N outside 0..nmax or a voxel index >= NV among an
// example's first N entries (block per example, grid-stride over examples).
__global__ void check_set(int64_t n_examples, int nmax, const uint16_t *set_vox, const int32_t *set_n, int *bad)
{
    for (int64_t ex = blockIdx.x; ex < n_examples; ex += gridDim.x) {
        const int nb = set_n[ex];
        if (nb < 0 || nb > nmax) {
            if (threadIdx.x == 0) *bad = 1;
            continue;
        }
        bool out = false;
        for (int j = threadIdx.x; j < nb; j += blockDim.x) out |= set_vox[ex * nmax + j] >= NV;
        if (out) *bad = 1;
    }
}

// MFMA B-operand tiles of a [n_out][128] weight matrix (the layout of NetDev):
// P[((tile*4 + kp)*64 + lane)*8 + j] = W[16 tile + lane%16][32 kp + 16 (j/4) + 4 (lane/16) + j%4]
__global__ void pack_b_tiles(int n_out, const bf16 *W, bf16 *P)
{
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)n_out * H) return;
    const int j = (int)(idx % 8), lane = (int)((idx / 8) % 64), kp = (int)((idx / 512) % 4);
    const int tile = (int)(idx / 2048);
    P[idx] = W[(size_t)(16 * tile + lane % 16) * H + 32 * kp + 16 * (j / 4) + 4 * (lane / 16) + j % 4];
}

// Voxel lists of walkers: vox[w][j] = voxel of particle j of walker w (the grid of
// the learned proposal over the class's gas region), n_out[w] = N.
__global__ void capture_voxels(int n_walkers, int stride, const ClassDev *cls, const int *walker_class,
                               const int32_t *n, const double *xyz, int xyz_stride, uint16_t *vox, int32_t *n_out)
{
    const int w = blockIdx.x;
    const ClassDev &C = cls[walker_class[w]];
    const int nw = n[w];
    const double gx = (double)kNetGrid / C.lx, gy = (double)kNetGrid / C.ly, gz = (double)kNetGrid / (C.zhi - C.zlo);
    for (int j = threadIdx.x; j < stride; j += blockDim.x) {
        int v = 0;
        if (j < nw) {
            const double *p = xyz + ((size_t)w * xyz_stride + j) * 3;
            int ix = (int)floor(p[0] * gx), iy = (int)floor(p[1] * gy), iz = (int)floor((p[2] - C.zlo) * gz);
            ix = ix < 0 ? 0 : (ix > kNetGrid - 1 ? kNetGrid - 1 : ix);
            iy = iy < 0 ? 0 : (iy > kNetGrid - 1 ? kNetGrid - 1 : iy);
            iz = iz < 0 ? 0 : (iz > kNetGrid - 1 ? kNetGrid - 1 : iz);
            v = (iz * kNetGrid + iy) * kNetGrid + ix;
        }
        vox[(size_t)w * stride + j] = (uint16_t)v;
    }
    if (threadIdx.x == 0) n_out[w] = nw;
}

// k-major copy of a [n_out][128] weight matrix: T[k][o] = W[o][k]
__global__ void transpose_kmajor(int n_out, const bf16 *W, bf16 *T)
{
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)n_out * H) return;
    const int k = (int)(idx / n_out), o = (int)(idx % n_out);
    T[idx] = W[(size_t)o * H + k];
}

}  // namespace mlpk
}  // namespace regc

using namespace regc;
using namespace regc::mlpk;

struct regc_mlp {
    int max_batch = 0, nmax = 0;
    hipStream_t stream = nullptr;
    DevBuf<float> p, g, m, v;
    DevBuf<bf16> p16;
    DevBuf<float> a1, a2, a3, logits, d32, dh, da, loss, ksplit;
    DevBuf<bf16> h1, h2, h3, d16, da16;
    DevBuf<uint16_t> bvox;
    DevBuf<int32_t> bn, bex, btgt;
    int64_t t = 0;   // Adam steps taken
    double ms_train = 0.0;
    int64_t steps_timed = 0;
};

static int mlp_workspace(regc_mlp *h, int B, int nmax)
{
    if (B <= h->max_batch && nmax <= h->nmax) return REGC_OK;
    const int Bm = std::max(B, h->max_batch), nm = std::max(nmax, h->nmax);
    int rc;
    if ((rc = h->a1.alloc((size_t)Bm * H)) || (rc = h->a2.alloc((size_t)Bm * H)) || (rc = h->a3.alloc((size_t)Bm * H)) ||
        (rc = h->logits.alloc((size_t)Bm * NV)) || (rc = h->d32.alloc((size_t)Bm * NV)) ||
        (rc = h->dh.alloc((size_t)Bm * H)) || (rc = h->da.alloc((size_t)Bm * H)) || (rc = h->loss.alloc(Bm)) ||
        (rc = h->h1.alloc((size_t)Bm * H)) || (rc = h->h2.alloc((size_t)Bm * H)) || (rc = h->h3.alloc((size_t)Bm * H)) ||
        (rc = h->d16.alloc((size_t)Bm * NV)) || (rc = h->da16.alloc((size_t)Bm * H)) ||
        (rc = h->bvox.alloc((size_t)Bm * nm)) || (rc = h->bn.alloc(Bm)) || (rc = h->bex.alloc(Bm)) ||
        (rc = h->btgt.alloc(Bm)) || (rc = h->ksplit.alloc((size_t)kSplitK * Bm * H)))
        return rc;
    h->max_batch = Bm;
    h->nmax = nm;
    return REGC_OK;
}

template <bool TA, bool TB, int EPI>
static hipError_t gemm(hipStream_t s, int M, int N, int K, const bf16 *A, int lda, const bf16 *B, int ldb, float *C,
                       int ldc, const float *bias = nullptr, bf16 *act = nullptr, int ldact = 0)
{
    hipLaunchKernelGGL((gemm_bf16<TA, TB, EPI>), dim3(N / 64, M / 64), dim3(256), 0, s, M, N, K, A, lda, B, ldb, C,
                       ldc, bias, act, ldact);
    return hipGetLastError();
}

// C [M][N] (ldc = N) of a long reduction (K a multiple of 16 * kSplitK): kSplitK
// partial products into the workspace, then their sum in a fixed order
template <bool TA, bool TB>
static hipError_t gemm_splitk(hipStream_t s, int M, int N, int K, const bf16 *A, int lda, const bf16 *B, int ldb,
                              float *C, float *work)
{
    hipLaunchKernelGGL((gemm_bf16<TA, TB, EPI_STORE>), dim3(N / 64, M / 64, kSplitK), dim3(256), 0, s, M, N, K, A, lda,
                       B, ldb, work, N, nullptr, nullptr, 0);
    const size_t count = (size_t)M * N;
    hipLaunchKernelGGL(sum_partials, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, kSplitK, count, work, C);
    return hipGetLastError();
}

// forward of the batch already in h->bvox/bn/bex (B a multiple of 64)
static int mlp_forward_dev(regc_mlp *h, int B, int nmax)
{
    hipStream_t s = h->stream;
    const bf16 *W1 = h->p16.p + OFF_W1, *W2 = h->p16.p + OFF_W2, *W3 = h->p16.p + OFF_W3, *W4 = h->p16.p + OFF_W4;
    const float *b1 = h->p.p + OFF_B1, *b2 = h->p.p + OFF_B2, *b3 = h->p.p + OFF_B3, *b4 = h->p.p + OFF_B4;
    hipLaunchKernelGGL(l1_forward, dim3(B), dim3(H), 0, s, nmax, h->bvox.p, h->bn.p, h->bex.p, W1, b1, h->a1.p, h->h1.p);
    REGC_HIP(hipGetLastError());
    REGC_HIP((gemm<false, true, EPI_BIAS_GELU>(s, B, H, H, h->h1.p, H, W2, H, h->a2.p, H, b2, h->h2.p, H)));
    REGC_HIP((gemm<false, true, EPI_BIAS_GELU>(s, B, H, H, h->h2.p, H, W3, H, h->a3.p, H, b3, h->h3.p, H)));
    REGC_HIP((gemm<false, true, EPI_BIAS>(s, B, NV, H, h->h3.p, H, W4, H, h->logits.p, NV, b4)));
    return REGC_OK;
}

// forward + backward of the batch in the workspace; gradients into h->g
static int mlp_backward_dev(regc_mlp *h, int B, int nmax)
{
    hipStream_t s = h->stream;
    int rc;
    if ((rc = mlp_forward_dev(h, B, nmax))) return rc;
    const bf16 *W2 = h->p16.p + OFF_W2, *W3 = h->p16.p + OFF_W3, *W4 = h->p16.p + OFF_W4;
    float *g = h->g.p;
    hipLaunchKernelGGL(softmax_xent, dim3(B), dim3(256), 0, s, B, h->logits.p, h->btgt.p, h->loss.p, h->d32.p, h->d16.p);
    REGC_HIP(hipGetLastError());
    // output layer: dW4 = d^T h3, db4 = colsum d, dh3 = d W4
    REGC_HIP((gemm<true, false, EPI_STORE>(s, NV, H, B, h->d16.p, NV, h->h3.p, H, g + OFF_W4, H)));
    hipLaunchKernelGGL(colsum, dim3(NV / 64), dim3(256), 0, s, B, NV, h->d32.p, g + OFF_B4);
    REGC_HIP(hipGetLastError());
    REGC_HIP((gemm_splitk<false, false>(s, B, H, NV, h->d16.p, NV, W4, H, h->dh.p, h->ksplit.p)));
    // hidden layers 3 and 2
    const int cnt = B * H, gb = (cnt + 255) / 256;
    hipLaunchKernelGGL(gelu_backward, dim3(gb), dim3(256), 0, s, cnt, h->dh.p, h->a3.p, h->da.p, h->da16.p);
    REGC_HIP(hipGetLastError());
    REGC_HIP((gemm<true, false, EPI_STORE>(s, H, H, B, h->da16.p, H, h->h2.p, H, g + OFF_W3, H)));
    hipLaunchKernelGGL(colsum, dim3(H / 64), dim3(256), 0, s, B, H, h->da.p, g + OFF_B3);
    REGC_HIP(hipGetLastError());
    REGC_HIP((gemm<false, false, EPI_STORE>(s, B, H, H, h->da16.p, H, W3, H, h->dh.p, H)));
    hipLaunchKernelGGL(gelu_backward, dim3(gb), dim3(256), 0, s, cnt, h->dh.p, h->a2.p, h->da.p, h->da16.p);
    REGC_HIP(hipGetLastError());
    REGC_HIP((gemm<true, false, EPI_STORE>(s, H, H, B, h->da16.p, H, h->h1.p, H, g + OFF_W2, H)));
    hipLaunchKernelGGL(colsum, dim3(H / 64), dim3(256), 0, s, B, H, h->da.p, g + OFF_B2);
    REGC_HIP(hipGetLastError());
    REGC_HIP((gemm<false, false, EPI_STORE>(s, B, H, H, h->da16.p, H, W2, H, h->dh.p, H)));
    // layer 1: gather's gradient is a scatter into the occupied voxels' columns
    hipLaunchKernelGGL(gelu_backward, dim3(gb), dim3(256), 0, s, cnt, h->dh.p, h->a1.p, h->da.p, h->da16.p);
    REGC_HIP(hipGetLastError());
    hipLaunchKernelGGL(colsum, dim3(H / 64), dim3(256), 0, s, B, H, h->da.p, g + OFF_B1);
    REGC_HIP(hipGetLastError());
    REGC_HIP(hipMemsetAsync(g + OFF_W1, 0, sizeof(float) * (size_t)NV * H, s));
    hipLaunchKernelGGL(l1_backward, dim3(B), dim3(H), 0, s, nmax, h->bvox.p, h->bn.p, h->bex.p, h->da.p, g + OFF_W1);
    REGC_HIP(hipGetLastError());
    return REGC_OK;
}

static int upload_batch(regc_mlp *h, int B, int nmax, const uint16_t *vox, const int32_t *n, const int32_t *excl,
                        const int32_t *target)
{
    hipStream_t s = h->stream;
    REGC_HIP(hipMemcpyAsync(h->bvox.p, vox, sizeof(uint16_t) * (size_t)B * nmax, hipMemcpyHostToDevice, s));
    REGC_HIP(hipMemcpyAsync(h->bn.p, n, sizeof(int32_t) * B, hipMemcpyHostToDevice, s));
    REGC_HIP(hipMemcpyAsync(h->bex.p, excl, sizeof(int32_t) * B, hipMemcpyHostToDevice, s));
    if (target) REGC_HIP(hipMemcpyAsync(h->btgt.p, target, sizeof(int32_t) * B, hipMemcpyHostToDevice, s));
    return REGC_OK;
}

static int check_batch(int B, int nmax, const uint16_t *vox, const int32_t *n, const int32_t *excl, const int32_t *target)
{
    REGC_CHECK(B > 0 && B % 64 == 0, REGC_EINVAL, "batch must be a positive multiple of 64");
    REGC_CHECK(nmax > 0 && nmax <= 65535, REGC_EINVAL, "bad nmax");
    for (int b = 0; b < B; ++b) {
        REGC_CHECK(n[b] >= 0 && n[b] <= nmax, REGC_EINVAL, "example %d: N out of range", b);
        REGC_CHECK(excl[b] >= -1 && excl[b] < std::max(n[b], 1), REGC_EINVAL, "example %d: bad left-out index", b);
        for (int j = 0; j < n[b]; ++j) REGC_CHECK(vox[(size_t)b * nmax + j] < NV, REGC_EINVAL, "voxel out of range");
        if (target) REGC_CHECK(target[b] >= 0 && target[b] < NV, REGC_EINVAL, "target voxel out of range");
    }
    return REGC_OK;
}

extern "C" int regc_mlp_create(const float *params, regc_mlp **out)
{
    REGC_CHECK(out, REGC_EINVAL, "null output pointer");
    regc_mlp *h = new regc_mlp();
    int rc;
    if ((rc = h->p.alloc(NPARAM)) || (rc = h->g.alloc(NPARAM)) || (rc = h->m.alloc(NPARAM)) ||
        (rc = h->v.alloc(NPARAM)) || (rc = h->p16.alloc(NPARAM)) || (rc = mlp_workspace(h, 64, 64))) {
        delete h;
        return rc;
    }
    if (params) {
        if (hipMemcpy(h->p.p, params, sizeof(float) * NPARAM, hipMemcpyHostToDevice) != hipSuccess) {
            delete h;
            set_error("hipMemcpy failed");
            return REGC_EHIP;
        }
    } else {
        (void)hipMemset(h->p.p, 0, sizeof(float) * NPARAM);
    }
    (void)hipMemset(h->m.p, 0, sizeof(float) * NPARAM);
    (void)hipMemset(h->v.p, 0, sizeof(float) * NPARAM);
    hipLaunchKernelGGL(to_bf16, dim3((unsigned)((NPARAM + 255) / 256)), dim3(256), 0, 0, (size_t)NPARAM, h->p.p, h->p16.p);
    if (hipDeviceSynchronize() != hipSuccess) {
        delete h;
        set_error("device synchronisation failed");
        return REGC_EHIP;
    }
    *out = h;
    return REGC_OK;
}

extern "C" int regc_mlp_param_count(int64_t *count)
{
    REGC_CHECK(count, REGC_EINVAL, "null argument");
    *count = (int64_t)NPARAM;
    return REGC_OK;
}

extern "C" int regc_mlp_set_stream(regc_mlp *h, void *stream)
{
    REGC_CHECK(h, REGC_EINVAL, "null handle");
    h->stream = (hipStream_t)stream;
    return REGC_OK;
}

extern "C" int regc_mlp_set_params(regc_mlp *h, const float *params)
{
    REGC_CHECK(h && params, REGC_EINVAL, "null argument");
    REGC_HIP(hipStreamSynchronize(h->stream));
    REGC_HIP(hipMemcpy(h->p.p, params, sizeof(float) * NPARAM, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(to_bf16, dim3((unsigned)((NPARAM + 255) / 256)), dim3(256), 0, h->stream, (size_t)NPARAM, h->p.p,
                       h->p16.p);
    REGC_HIP(hipGetLastError());
    REGC_HIP(hipMemsetAsync(h->m.p, 0, sizeof(float) * NPARAM, h->stream));
    REGC_HIP(hipMemsetAsync(h->v.p, 0, sizeof(float) * NPARAM, h->stream));
    h->t = 0;
    REGC_HIP(hipStreamSynchronize(h->stream));
    return REGC_OK;
}

extern "C" int regc_mlp_get_params(regc_mlp *h, float *params)
{
    REGC_CHECK(h && params, REGC_EINVAL, "null argument");
    REGC_HIP(hipStreamSynchronize(h->stream));
    REGC_HIP(hipMemcpy(params, h->p.p, sizeof(float) * NPARAM, hipMemcpyDeviceToHost));
    return REGC_OK;
}

extern "C" int regc_mlp_forward(regc_mlp *h, int B, int nmax, const uint16_t *vox, const int32_t *n,
                                const int32_t *excl, float *logits)
{
    REGC_CHECK(h && vox && n && excl && logits, REGC_EINVAL, "null argument");
    int rc;
    if ((rc = check_batch(B, nmax, vox, n, excl, nullptr)) || (rc = mlp_workspace(h, B, nmax)) ||
        (rc = upload_batch(h, B, nmax, vox, n, excl, nullptr)) || (rc = mlp_forward_dev(h, B, nmax)))
        return rc;
    REGC_HIP(hipStreamSynchronize(h->stream));
    REGC_HIP(hipMemcpy(logits, h->logits.p, sizeof(float) * (size_t)B * NV, hipMemcpyDeviceToHost));
    return REGC_OK;
}

extern "C" int regc_mlp_loss_grads(regc_mlp *h, int B, int nmax, const uint16_t *vox, const int32_t *n,
                                   const int32_t *excl, const int32_t *target, double *loss, float *grads)
{
    REGC_CHECK(h && vox && n && excl && target, REGC_EINVAL, "null argument");
    int rc;
    if ((rc = check_batch(B, nmax, vox, n, excl, target)) || (rc = mlp_workspace(h, B, nmax)) ||
        (rc = upload_batch(h, B, nmax, vox, n, excl, target)) || (rc = mlp_backward_dev(h, B, nmax)))
        return rc;
    REGC_HIP(hipStreamSynchronize(h->stream));
    if (loss) {
        std::vector<float> l(B);
        REGC_HIP(hipMemcpy(l.data(), h->loss.p, sizeof(float) * B, hipMemcpyDeviceToHost));
        double s = 0.0;
        for (float x : l) s += x;
        *loss = s / B;
    }
    if (grads) REGC_HIP(hipMemcpy(grads, h->g.p, sizeof(float) * NPARAM, hipMemcpyDeviceToHost));
    return REGC_OK;
}

extern "C" int regc_mlp_step(regc_mlp *h, int B, int nmax, const uint16_t *vox, const int32_t *n,
                             const int32_t *excl, const int32_t *target, double lr, double *loss, float *grads)
{
    REGC_CHECK(h && vox && n && excl && target, REGC_EINVAL, "null argument");
    REGC_CHECK(lr > 0, REGC_EINVAL, "learning rate must be positive");
    int rc;
    if ((rc = check_batch(B, nmax, vox, n, excl, target)) || (rc = mlp_workspace(h, B, nmax)) ||
        (rc = upload_batch(h, B, nmax, vox, n, excl, target)) || (rc = mlp_backward_dev(h, B, nmax)))
        return rc;
    hipStream_t s = h->stream;
    const float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
    h->t += 1;
    const float c1 = 1.0f - powf(beta1, (float)h->t), c2 = 1.0f - powf(beta2, (float)h->t);
    hipLaunchKernelGGL(adam_update, dim3((unsigned)((NPARAM + 255) / 256)), dim3(256), 0, s, (size_t)NPARAM, h->p.p,
                       h->g.p, h->m.p, h->v.p, (float)lr, c1, c2, beta1, beta2, eps, h->p16.p);
    REGC_HIP(hipGetLastError());
    REGC_HIP(hipStreamSynchronize(s));
    if (loss) {
        std::vector<float> l(B);
        REGC_HIP(hipMemcpy(l.data(), h->loss.p, sizeof(float) * B, hipMemcpyDeviceToHost));
        double acc = 0.0;
        for (float x : l) acc += x;
        *loss = acc / B;
    }
    if (grads) REGC_HIP(hipMemcpy(grads, h->g.p, sizeof(float) * NPARAM, hipMemcpyDeviceToHost));
    return REGC_OK;
}

extern "C" int regc_mlp_train(regc_mlp *h, int64_t n_examples, int nmax, const uint16_t *vox_dev,
                              const int32_t *n_dev, int64_t steps, int batch, double lr, uint64_t seed,
                              double *mean_loss)
{
    REGC_CHECK(h && vox_dev && n_dev, REGC_EINVAL, "null argument");
    REGC_CHECK(n_examples > 0 && steps > 0 && lr > 0, REGC_EINVAL, "bad training size");
    REGC_CHECK(batch > 0 && batch % 64 == 0, REGC_EINVAL, "batch must be a positive multiple of 64");
    REGC_CHECK(nmax > 0 && nmax <= 65535, REGC_EINVAL, "bad nmax");
    int rc;
    if ((rc = mlp_workspace(h, batch, nmax))) return rc;
    hipStream_t s = h->stream;
    DevBuf<float> lsum;
    DevBuf<int> bad;
    if ((rc = lsum.alloc(batch)) || (rc = bad.alloc(1))) return rc;
    {
        // the batch kernels index by N and gather W1 rows by voxel: check the set first
        int h_bad = 0;
        REGC_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), s));
        hipLaunchKernelGGL(check_set, dim3((unsigned)std::min<int64_t>(n_examples, 4096)), dim3(64), 0, s, n_examples,
                           nmax, vox_dev, n_dev, bad.p);
        REGC_HIP(hipGetLastError());
        REGC_HIP(hipMemcpyAsync(&h_bad, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
        REGC_HIP(hipStreamSynchronize(s));
        REGC_CHECK(!h_bad, REGC_EINVAL, "training set: an N outside 0..%d or a voxel index >= %d", nmax, NV);
    }
    ScopedEvent e0, e1;
    REGC_HIP(e0.create());
    REGC_HIP(e1.create());
    REGC_HIP(hipEventRecord(e0.e, s));
    const float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
    double loss_acc = 0.0;
    std::vector<float> lh(batch);
    for (int64_t st = 0; st < steps; ++st) {
        hipLaunchKernelGGL(make_batch, dim3(batch), dim3(64), 0, s, batch, nmax, n_examples, vox_dev, n_dev,
                           h->t, (uint32_t)seed, (uint32_t)(seed >> 32), h->bvox.p, h->bn.p, h->bex.p, h->btgt.p);
        REGC_HIP(hipGetLastError());
        if ((rc = mlp_backward_dev(h, batch, nmax))) return rc;
        h->t += 1;
        const float c1 = 1.0f - powf(beta1, (float)h->t), c2 = 1.0f - powf(beta2, (float)h->t);
        hipLaunchKernelGGL(adam_update, dim3((unsigned)((NPARAM + 255) / 256)), dim3(256), 0, s, (size_t)NPARAM, h->p.p,
                           h->g.p, h->m.p, h->v.p, (float)lr, c1, c2, beta1, beta2, eps, h->p16.p);
        REGC_HIP(hipGetLastError());
        if (mean_loss && (st == steps - 1 || (st + 1) % 50 == 0)) {
            REGC_HIP(hipMemcpyAsync(lh.data(), h->loss.p, sizeof(float) * batch, hipMemcpyDeviceToHost, s));
            REGC_HIP(hipStreamSynchronize(s));
            double a = 0.0;
            for (float x : lh) a += x;
            loss_acc = a / batch;
        }
    }
    REGC_HIP(hipEventRecord(e1.e, s));
    REGC_HIP(hipEventSynchronize(e1.e));
    float ms = 0.f;
    REGC_HIP(hipEventElapsedTime(&ms, e0.e, e1.e));
    h->ms_train += ms;
    h->steps_timed += steps;
    if (mean_loss) *mean_loss = loss_acc;
    return REGC_OK;
}

namespace regc {
hipError_t launch_capture_voxels(int n_walkers, int stride, const ClassDev *cls, const int *walker_class,
                                 const int32_t *n, const double *xyz, int xyz_stride, uint16_t *vox, int32_t *n_out,
                                 hipStream_t s)
{
    hipLaunchKernelGGL(capture_voxels, dim3(n_walkers), dim3(64), 0, s, n_walkers, stride, cls, walker_class, n, xyz,
                       xyz_stride, vox, n_out);
    return hipGetLastError();
}

int mlp_export_sampler(regc_mlp *h, bool kmajor, uint16_t *w1, uint16_t *w2, uint16_t *w3, uint16_t *w4, float *b1,
                       float *b2, float *b3, float *b4, hipStream_t s)
{
    REGC_CHECK(h, REGC_EINVAL, "null network");
    REGC_HIP(hipStreamSynchronize(h->stream));
    REGC_HIP(hipMemcpyAsync(w1, h->p16.p + OFF_W1, sizeof(bf16) * (size_t)NV * H, hipMemcpyDeviceToDevice, s));
    const bf16 *src[3] = {h->p16.p + OFF_W2, h->p16.p + OFF_W3, h->p16.p + OFF_W4};
    uint16_t *dst[3] = {w2, w3, w4};
    const int n_out[3] = {H, H, NV};
    for (int q = 0; q < 3; ++q) {
        const unsigned blocks = (unsigned)((size_t)n_out[q] * H / 256);
        if (kmajor)
            hipLaunchKernelGGL(transpose_kmajor, dim3(blocks), dim3(256), 0, s, n_out[q], src[q], dst[q]);
        else
            hipLaunchKernelGGL(pack_b_tiles, dim3(blocks), dim3(256), 0, s, n_out[q], src[q], dst[q]);
        REGC_HIP(hipGetLastError());
    }
    REGC_HIP(hipMemcpyAsync(b1, h->p.p + OFF_B1, sizeof(float) * H, hipMemcpyDeviceToDevice, s));
    REGC_HIP(hipMemcpyAsync(b2, h->p.p + OFF_B2, sizeof(float) * H, hipMemcpyDeviceToDevice, s));
    REGC_HIP(hipMemcpyAsync(b3, h->p.p + OFF_B3, sizeof(float) * H, hipMemcpyDeviceToDevice, s));
    REGC_HIP(hipMemcpyAsync(b4, h->p.p + OFF_B4, sizeof(float) * NV, hipMemcpyDeviceToDevice, s));
    return REGC_OK;
}
}  // namespace regc

extern "C" int regc_mlp_timing(regc_mlp *h, double *ms, int64_t *steps)
{
    REGC_CHECK(h, REGC_EINVAL, "null handle");
    if (ms) *ms = h->ms_train;
    if (steps) *steps = h->steps_timed;
    return REGC_OK;
}

extern "C" void regc_mlp_destroy(regc_mlp *h) { delete h; }
