// swap_dev.h -- the replica-exchange step of one class as a device function, shared by
// the exchange kernel and the persistent sweep launch (arXiv:1908.11118, Sec. II.A.2;
// the pair schemes and the acceptance are described in swap.hip).
#pragma once
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

// Loads and counter updates of the exchange.  COHERENT (a workgroup of the persistent
// sweep launch, which reads what other workgroups wrote during the same launch):
// device-scope loads that skip the compute unit's L1, device-scope atomic counters.
template <bool COHERENT, typename T>
__device__ __forceinline__ T xload(const T *p)
{
    if (COHERENT) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return *p;
}

template <bool COHERENT>
__device__ __forceinline__ void xcount(unsigned long long *p)
{
    if (COHERENT) atomicAdd(p, 1ull);
    else *p += 1ull;
}

// Exchange step q of class c: threads tid, tid + nthr, ... take the pairs.
template <bool COHERENT>
__device__ void swap_class(const SwapArgs &a, int c, int64_t q, int tid, int nthr)
{
    const ClassDev &C = a.cls[c];
    const int L = C.n_t, M = C.n_mu, off = C.state_off;
    const uint32_t stream = 0xFFFFFFFFu - (uint32_t)c;
    const uint4 T = philox4x32_10(make_uint4(0u, (uint32_t)q, stream, 3u), a.key0, a.key1);
    const int type = (int)(T.x >> 30);
    // scheme 1: origin of the 2x2 blocks, so that blocks of both tilings alternate
    const int ol = a.scheme == 1 ? (int)((T.x >> 29) & 1u) : 0;
    const int om = a.scheme == 1 ? (int)((T.x >> 28) & 1u) : 0;
    const int P = pair_count(a.scheme, type, ol, om, L, M);
    for (int p = tid; p < P; p += nthr) {
        int sa, sb;
        pair_of(a.scheme, type, ol, om, p, L, M, sa, sb);
        const int lo = sa < sb ? sa : sb;
        const uint4 R = philox4x32_10(make_uint4((uint32_t)lo, (uint32_t)q, stream, 4u), a.key0, a.key1);
        const int ga = off + sa, gb = off + sb;
        const int i = xload<COHERENT>(a.wos + ga), j = xload<COHERENT>(a.wos + gb);
        const double x = (a.beta[ga] - a.beta[gb]) * (xload<COHERENT>(a.e + i) - xload<COHERENT>(a.e + j)) +
                         (double)(xload<COHERENT>(a.n + j) - xload<COHERENT>(a.n + i)) * (a.lnz[ga] - a.lnz[gb]);
        xcount<COHERENT>(a.att + (size_t)type * a.S_total + off + lo);
        if (metropolis(x, uniform53(R.x, R.y))) {
            a.label[i] = sb;
            a.label[j] = sa;
            a.wos[ga] = j;
            a.wos[gb] = i;
            xcount<COHERENT>(a.acc + (size_t)type * a.S_total + off + lo);
        }
    }
}

}  // namespace regc
