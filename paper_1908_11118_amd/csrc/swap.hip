// swap.hip -- the replica-exchange step (arXiv:1908.11118, Sec. II.A.2).
//
// One of four collective neighbour-swap types is drawn with probability 1/4 and
// every disjoint pair of that type is attempted independently.  Scheme 0: even
// T-axis pairs (2a, 2a+1), odd T-axis pairs (2a+1, 2a+2), even and odd mu-axis
// pairs.  Scheme 1: inside 2x2 blocks of the grid, pairs along T, along mu, and
// along the two diagonals; the blocks start at (ol + 2a, om + 2b), the origin
// (ol, om) in {0,1}^2 drawn with the type (bits 29 and 28 of its word), so the even
// and odd tilings alternate and a configuration can cross the grid.  The pair acceptance is the ratio of the GC densities
// (Eq. (1)) of both walkers in both states, i.e. Eq. (6) read as
//     ln A = (beta_a - beta_b)(E_i - E_j) + (N_j - N_i)(ln z_a - ln z_b)
// for walker i in state a and walker j in state b.  Labels are permuted; the
// configurations stay where they are.  One workgroup per class; one lane per pair.
#include "regc_dev.h"
#include "philox_dev.h"

namespace regc {

__device__ __forceinline__ void pair_of(int scheme, int type, int ol, int om, int p, int L, int M, int &sa, int &sb)
{
    if (scheme == 0) {
        if (type < 2) {
            const int a = p / M, m = p - a * M;
            sa = (type + 2 * a) * M + m;
            sb = sa + M;
        } else {
            const int o = type - 2;
            const int B = (M - o) / 2;
            const int l = p / B, bb = p - l * B;
            sa = l * M + o + 2 * bb;
            sb = sa + 1;
        }
    } else {
        const int bm = (M - om) / 2;
        const int per = type < 2 ? 2 : 1;
        const int blk = p / per, k = p - blk * per;
        const int l = ol + 2 * (blk / bm), m = om + 2 * (blk - (blk / bm) * bm);
        const int s00 = l * M + m, s01 = s00 + 1, s10 = s00 + M, s11 = s10 + 1;
        if (type == 0) { sa = k ? s01 : s00; sb = k ? s11 : s10; }
        else if (type == 1) { sa = k ? s10 : s00; sb = k ? s11 : s01; }
        else if (type == 2) { sa = s00; sb = s11; }
        else { sa = s01; sb = s10; }
    }
}

__device__ __forceinline__ int pair_count(int scheme, int type, int ol, int om, int L, int M)
{
    if (scheme == 0) {
        if (type < 2) return ((L - type) / 2) * M;
        return L * ((M - (type - 2)) / 2);
    }
    return (type < 2 ? 2 : 1) * ((L - ol) / 2) * ((M - om) / 2);
}

__global__ void __launch_bounds__(256) swap_kernel(SwapArgs a)
{
    const int c = blockIdx.x;
    const ClassDev &C = a.cls[c];
    const int L = C.n_t, M = C.n_mu, off = C.state_off;
    const uint32_t stream = 0xFFFFFFFFu - (uint32_t)c;
    const int64_t q = a.clock ? (a.clock[0] + a.interval) / a.swap_every - 1 : a.q;
    const uint4 T = philox4x32_10(make_uint4(0u, (uint32_t)q, stream, 3u), a.key0, a.key1);
    const int type = (int)(T.x >> 30);
    // scheme 1: origin of the 2x2 blocks, so that blocks of both tilings alternate
    const int ol = a.scheme == 1 ? (int)((T.x >> 29) & 1u) : 0;
    const int om = a.scheme == 1 ? (int)((T.x >> 28) & 1u) : 0;
    const int P = pair_count(a.scheme, type, ol, om, L, M);
    for (int p = threadIdx.x; p < P; p += blockDim.x) {
        int sa, sb;
        pair_of(a.scheme, type, ol, om, p, L, M, sa, sb);
        const int lo = sa < sb ? sa : sb;
        const uint4 R = philox4x32_10(make_uint4((uint32_t)lo, (uint32_t)q, stream, 4u), a.key0, a.key1);
        const int ga = off + sa, gb = off + sb;
        const int i = a.wos[ga], j = a.wos[gb];
        const double x = (a.beta[ga] - a.beta[gb]) * (a.e[i] - a.e[j]) +
                         (double)(a.n[j] - a.n[i]) * (a.lnz[ga] - a.lnz[gb]);
        a.att[(size_t)type * a.S_total + off + lo] += 1ull;
        if (metropolis(x, uniform53(R.x, R.y))) {
            a.label[i] = sb;
            a.label[j] = sa;
            a.wos[ga] = j;
            a.wos[gb] = i;
            a.acc[(size_t)type * a.S_total + off + lo] += 1ull;
        }
    }
}

// Advances the device-side sweep clock after one replayed exchange interval.
__global__ void clock_advance(int64_t *clock, int n)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) clock[0] += n;
}

hipError_t launch_clock_advance(int64_t *clock, int n, hipStream_t s)
{
    hipLaunchKernelGGL(clock_advance, dim3(1), dim3(64), 0, s, clock, n);
    return hipGetLastError();
}

__global__ void clock_set(int64_t *clock, int64_t value)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) clock[0] = value;
}

hipError_t launch_clock_set(int64_t *clock, int64_t value, hipStream_t s)
{
    hipLaunchKernelGGL(clock_set, dim3(1), dim3(64), 0, s, clock, value);
    return hipGetLastError();
}

hipError_t launch_swap(const SwapArgs &a, int n_class, hipStream_t s)
{
    hipLaunchKernelGGL(swap_kernel, dim3(n_class), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace regc
