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

hipError_t launch_observables(const ObsArgs &a, hipStream_t s)
{
    if (a.n_obs > kObsMaxBins) return hipErrorInvalidValue;
    hipLaunchKernelGGL(obs_kernel, dim3(a.n_walkers), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace regc
