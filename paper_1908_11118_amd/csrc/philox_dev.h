// philox_dev.h -- counter-based random numbers for the REGC kernels.
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As Easy
// as 1, 2, 3", SC'11): ten rounds of two 32x32->64-bit multiplications (by
// 0xD2511F53 and 0xCD9E8D57) with a Feistel-like word permutation; the 64-bit
// key is advanced by the Weyl increments 0x9E3779B9 / 0xBB67AE85 between rounds.
//
// Stream layout (identical trajectories need identical words):
//   trial t of sweep s of walker w:  counter (t, s, w, 0) -> A0..A3,
//                                    counter (t, s, w, 1) -> B0..B3
//     A0 move type, A1 particle index floor(A1*N/2^32), A2 A3 B0 coordinates,
//     B1 B2 the 53-bit acceptance uniform, B3 spare;
//   exchange step q of class c:      counter (0, q, 0xFFFFFFFF - c, 3) -> type = word0 >> 30
//   pair with lower state p:         counter (p, q, 0xFFFFFFFF - c, 4) -> word0, word1 uniform
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace regc {

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi_a = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo_a = 0xD2511F53u * c.x;
        const uint32_t hi_b = __umulhi(0xCD9E8D57u, c.z);
        const uint32_t lo_b = 0xCD9E8D57u * c.z;
        c = make_uint4(hi_b ^ c.y ^ k0, lo_b, hi_a ^ c.w ^ k1, lo_a);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// (w + 1/2) / 2^32: exact in FP64, strictly inside (0, 1)
__device__ __forceinline__ double uniform_open(uint32_t w)
{
    return ((double)w + 0.5) * (1.0 / 4294967296.0);
}

// 53-bit uniform in [0, 1) from two words, exact in FP64
__device__ __forceinline__ double uniform53(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

// Metropolis: accept when x = ln(ratio) >= 0, else when U < exp(x)
__device__ __forceinline__ bool metropolis(double x, double U)
{
    return x >= 0.0 || U < exp(x);
}

}  // namespace regc
