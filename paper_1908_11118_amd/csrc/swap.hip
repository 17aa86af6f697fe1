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
#include "swap_dev.h"

namespace regc {

__global__ void __launch_bounds__(256) swap_kernel(SwapArgs a)
{
    const int64_t q = a.clock ? (a.clock[0] + a.interval) / a.swap_every - 1 : a.q;
    swap_class<false>(a, blockIdx.x, q, threadIdx.x, blockDim.x);
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

// Walker order of a sweep launch, one workgroup per class: the class's walkers are
// ranked by their current particle count (the cost of their trials; counts bucketed
// into 64 ranges, descending, ties in arrival order) and dealt round-robin to the
// class's workgroups, rank r to workgroup r mod nb, slot r / nb.  Every workgroup
// then holds walkers from the whole range of costs, instead of neighbouring states
// of the grid with similar particle counts, and the compute units finish together.
// Within a workgroup whose size is a multiple of four, the slots go to the waves in
// rows of four, every other row reversed: the waves of a workgroup are spread over
// the compute unit's four SIMDs in turn, so each SIMD pairs a costly walker with a
// cheap one (config 3: 11.03 -> 10.89 ms per launch).
// Classes whose walker count is not a multiple of the workgroup size keep the
// identity order.  The order decides only which wave runs which walker: every
// walker's trials, random numbers and results are the same in any order.
__global__ void __launch_bounds__(1024) balance_kernel(const ClassDev *cls, const int32_t *n, int wpb, int *wslot)
{
    constexpr int kBuckets = 64;
    __shared__ int start[kBuckets];
    const ClassDev &C = cls[blockIdx.x];
    const int off = C.walker_off, S = C.n_walkers, nv = C.n_max + 1;
    if (S % wpb != 0) {
        for (int k = threadIdx.x; k < S; k += blockDim.x) wslot[off + k] = off + k;
        return;
    }
    auto bucket = [&](int v) {
        v = v < 0 ? 0 : (v >= nv ? nv - 1 : v);
        return (int)(((int64_t)v * kBuckets) / nv);
    };
    if (threadIdx.x < kBuckets) start[threadIdx.x] = 0;
    __syncthreads();
    for (int k = threadIdx.x; k < S; k += blockDim.x) atomicAdd(&start[bucket(n[off + k])], 1);
    __syncthreads();
    if (threadIdx.x < kBuckets) {
        // walkers in buckets above this one: suffix sums over the 64 lanes
        const int lane = threadIdx.x;
        const int h = start[lane];
        int s = h;
#pragma unroll
        for (int o = 1; o < kBuckets; o <<= 1) {
            const int t = __shfl_down(s, o);
            s += lane + o < kBuckets ? t : 0;
        }
        start[lane] = s - h;
    }
    __syncthreads();
    const int nb = S / wpb;
    const bool snake = wpb % 4 == 0;
    for (int k = threadIdx.x; k < S; k += blockDim.x) {
        const int r = atomicAdd(&start[bucket(n[off + k])], 1);
        const int s = r / nb, row = s >> 2, col = s & 3;
        const int p = snake && (row & 1) ? 4 * row + 3 - col : s;
        wslot[off + (r % nb) * wpb + p] = off + k;
    }
}

hipError_t launch_balance(const ClassDev *cls, int n_class, const int32_t *n, int wpb, int *wslot, hipStream_t s)
{
    hipLaunchKernelGGL(balance_kernel, dim3(n_class), dim3(1024), 0, s, cls, n, wpb, wslot);
    return hipGetLastError();
}

hipError_t launch_swap(const SwapArgs &a, int n_class, hipStream_t s)
{
    hipLaunchKernelGGL(swap_kernel, dim3(n_class), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace regc
