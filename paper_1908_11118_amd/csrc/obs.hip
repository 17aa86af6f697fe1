// obs.hip -- structural observables of every walker at a sample point (the axial
// density and the lateral radial distribution of a layer, Sec. III.A), as integer
// counts per sample for the reweighting of Eq. (11).  One wavefront per walker,
// histograms in LDS.  Compiled without FP contraction: the bin of every particle
// and pair is the one a plain FP64 evaluation gives (minimum image by comparison
// with half the box, r = sqrt(dx^2 + dy^2), bin = floor(r / dr)).
#include "regc_dev.h"

namespace regc {

constexpr int kObsMaxBins = 2048;

__device__ __forceinline__ double obs_min_image(double d, double box)
{
    return d > 0.5 * box ? d - box : (d < -0.5 * box ? d + box : d);
}

__global__ void __launch_bounds__(64) obs_kernel(ObsArgs a)
{
    __shared__ uint32_t hist[kObsMaxBins];
    const int w = blockIdx.x, lane = threadIdx.x;
    const ClassDev &C = a.cls[a.walker_class[w]];
    const int n = a.n[w];
    const double *x = a.xyz + (size_t)w * a.xyz_stride * 3;
    for (int k = lane; k < a.n_obs; k += 64) hist[k] = 0u;
    __syncthreads();
    const int nz = (int)ceil((C.zhi - C.zlo) / a.dz);
    uint32_t in_layer = 0;
    for (int i = lane; i < n; i += 64) {
        const double z = x[3 * i + 2];
        int kz = (int)floor((z - C.zlo) / a.dz);
        kz = kz < 0 ? 0 : (kz > nz - 1 ? nz - 1 : kz);
        atomicAdd(hist + kz, 1u);
        in_layer += (z >= a.layer_lo && z < a.layer_hi) ? 1u : 0u;
    }
    for (int i = 0; i < n; ++i) {
        const double zi = x[3 * i + 2];
        if (!(zi >= a.layer_lo && zi < a.layer_hi)) continue;       // uniform across the wave
        const double xi = x[3 * i], yi = x[3 * i + 1];
        for (int j = i + 1 + lane; j < n; j += 64) {
            const double zj = x[3 * j + 2];
            if (!(zj >= a.layer_lo && zj < a.layer_hi)) continue;
            const double dx = obs_min_image(xi - x[3 * j], C.lx);
            const double dy = obs_min_image(yi - x[3 * j + 1], C.ly);
            const double r = sqrt(dx * dx + dy * dy);
            const int kr = (int)floor(r / a.dr);
            if (kr < a.n_r) atomicAdd(hist + a.n_z + kr, 1u);
        }
    }
    atomicAdd(hist + a.n_z + a.n_r, in_layer);
    __syncthreads();
    uint32_t *out = a.out + (size_t)w * a.n_obs;
    for (int k = lane; k < a.n_obs; k += 64) out[k] = hist[k];
}

// IEEE double -> unsigned key of the same order (zero of either sign as +0)
__device__ __forceinline__ unsigned long long energy_key(double e)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(e == 0.0 ? 0.0 : e);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__device__ __forceinline__ unsigned long long load_u64(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int load_i32(const int *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One workgroup: (0) remember the keys, (1) atomic minimum of every walker's energy
// key per (class, N), (2) among walkers at a new strict minimum the lowest index,
// (3) that walker stores its energy and configuration; the index slots are cleared.
// The result is the oracle's sequential rule (walkers in index order, replaced only
// by a strictly lower energy).
__global__ void __launch_bounds__(1024) minima_kernel(MinArgs a)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const int slots = a.n_class * a.nN;
    for (int k = tid; k < slots; k += nt) a.old_key[k] = load_u64(a.key + k);
    __syncthreads();
    for (int w = tid; w < a.n_walkers; w += nt)
        atomicMin(a.key + a.walker_class[w] * a.nN + a.n[w], energy_key(a.e[w]));
    __syncthreads();
    for (int w = tid; w < a.n_walkers; w += nt) {
        const int k = a.walker_class[w] * a.nN + a.n[w];
        const unsigned long long ek = energy_key(a.e[w]);
        if (ek == load_u64(a.key + k) && ek < a.old_key[k]) atomicMin(a.widx + k, w);
    }
    __syncthreads();
    for (int w = tid; w < a.n_walkers; w += nt) {
        const int k = a.walker_class[w] * a.nN + a.n[w];
        if (load_i32(a.widx + k) != w) continue;
        a.e_min[k] = a.e[w];
        const double *src = a.xyz + (size_t)w * a.xyz_stride * 3;
        double *dst = a.xyz_min + (size_t)k * a.xyz_stride * 3;
        for (int q = 0; q < 3 * a.n[w]; ++q) dst[q] = src[q];
    }
    __syncthreads();
    for (int w = tid; w < a.n_walkers; w += nt) {
        const int k = a.walker_class[w] * a.nN + a.n[w];
        if (load_i32(a.widx + k) == w) a.widx[k] = 0x7fffffff;
    }
}

hipError_t launch_minima(const MinArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(minima_kernel, dim3(1), dim3(1024), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_observables(const ObsArgs &a, hipStream_t s)
{
    if (a.n_obs > kObsMaxBins) return hipErrorInvalidValue;
    hipLaunchKernelGGL(obs_kernel, dim3(a.n_walkers), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace regc
