// sweep.hip -- the REGC sweep kernel: K grand-canonical / displacement trials per
// sweep for every walker, one wavefront (64 lanes) per walker, its gas
// coordinates and its class's frozen slab resident in LDS for the whole launch.
//
// This file is compiled twice:
//   -DREGC_FP64 with -ffp-contract=off : every operation in FP64 (trajectory-parity
//                                        mode; the same decisions as a sequential
//                                        FP64 reference up to summation order and exp);
//   -DREGC_FP32                        : pair terms and their per-lane sums in FP32,
//                                        running energy, acceptance test in FP64.
//
// Per trial (arXiv:1908.11118, Sec. II.A.1 and II.A.3):
//   move type from word A0 (displacement / insertion / removal, thresholds set
//   from p_disp, p_ins); the affected particle i = floor(A1 * N / 2^32);
//   displacement by a uniform vector in the cube [-d, d]^3, Eq. (7): ln A = -beta dE;
//   insertion at a uniform point of V, Eq. (3) with the exponent read as
//   beta [mu - (E_{N+1} - E_N)]: ln A = ln z + ln V - ln(N+1) - beta dE;
//   removal, Eq. (2): ln A = ln N - ln z - ln V - beta dE;
//   accept when ln A >= 0 or U53 < exp(ln A).
// dE is the sum of LJ pair terms of the moved particle over the other gas atoms
// (lanes stride over them) and over the slab atoms (all of them, or the 3x3
// stencil of x-y columns around the particle), reduced across the wave.
// Storage rule: insertion appends, removal moves the last particle into the
// freed slot.
#include "regc_dev.h"
#include "philox_dev.h"

namespace regc {

#if defined(REGC_FP64)
typedef double Real;
struct alignas(32) Real4 { double x, y, z, w; };
#define SWEEP_KERNEL sweep_kernel_f64
#define SWEEP_LAUNCH launch_sweep_f64
#define ENERGY_KERNEL energy_kernel_f64
#define ENERGY_LAUNCH launch_energy_f64
#elif defined(REGC_FP32)
typedef float Real;
struct alignas(16) Real4 { float x, y, z, w; };
#define SWEEP_KERNEL sweep_kernel_f32
#define SWEEP_LAUNCH launch_sweep_f32
#define ENERGY_KERNEL energy_kernel_f32
#define ENERGY_LAUNCH launch_energy_f32
#else
#error "compile with -DREGC_FP64 or -DREGC_FP32"
#endif

struct Box {
    Real lx, ly, hx, hy, ix, iy;
};

__device__ __forceinline__ Real min_image(Real d, Real L, Real half, Real inv)
{
#if defined(REGC_FP64)
    (void)inv;
    return d > half ? d - L : (d < -half ? d + L : d);
#else
    (void)half;
    return d - L * rintf(d * inv);
#endif
}

__device__ __forceinline__ Real dist2(const Box &b, Real px, Real py, Real pz, const Real4 &q)
{
    const Real dx = min_image(px - q.x, b.lx, b.hx, b.ix);
    const Real dy = min_image(py - q.y, b.ly, b.hy, b.iy);
    const Real dz = pz - q.z;
    return dx * dx + dy * dy + dz * dz;
}

struct Pair {
    Real sig2, eps4, shift, rc2, hc2;
};

__device__ __forceinline__ Real lj(Real r2, const Pair &p)
{
#if defined(REGC_FP64)
    const double s2 = p.sig2 / r2;
#else
    const float s2 = p.sig2 * __builtin_amdgcn_rcpf(r2);
#endif
    const Real s6 = s2 * s2 * s2;
    const Real v = p.eps4 * (s6 * s6 - s6) - p.shift;
    return r2 < p.rc2 ? v : Real(0);
}

__device__ __forceinline__ Real wave_sum(Real v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t bcast(uint32_t v, int lane)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

// Slab access: all atoms, or the 3x3 column stencil around (cx, cy).
struct SlabView {
    const Real4 *atoms;
    const int16_t *stencil;   // [ncol][9]
    int len;                  // entries when unbinned
    int bins, ncx, ncy, cap;
    float inv_cap;
    Real inv_cw_x, inv_cw_y;
    Real top_plus_rc;
};

__device__ __forceinline__ int column_of(const SlabView &sv, Real x, Real y)
{
    int cx = (int)(x * sv.inv_cw_x);
    int cy = (int)(y * sv.inv_cw_y);
    cx = cx < 0 ? 0 : (cx >= sv.ncx ? sv.ncx - 1 : cx);
    cy = cy < 0 ? 0 : (cy >= sv.ncy ? sv.ncy - 1 : cy);
    return cy * sv.ncx + cx;
}

// Sum over slab candidates of lj(p) (and of lj(q) when TWO), lanes striding.
template <bool TWO>
__device__ __forceinline__ void slab_terms(const SlabView &sv, const Box &b, const Pair &pp, int lane,
                                           Real px, Real py, Real pz, Real qx, Real qy, Real qz,
                                           Real cxp, Real cyp, Real &acc_p, Real &acc_q, bool &core)
{
    if (!sv.bins) {
        for (int k = lane; k < sv.len; k += kWave) {
            const Real4 a = sv.atoms[k];
            const Real r2 = dist2(b, px, py, pz, a);
            core |= r2 < pp.hc2;
            acc_p += lj(r2, pp);
            if (TWO) acc_q += lj(dist2(b, qx, qy, qz, a), pp);
        }
    } else {
        const int16_t *st = sv.stencil + column_of(sv, cxp, cyp) * 9;
        const int total = 9 * sv.cap;
        for (int k = lane; k < total; k += kWave) {
            const int sp = (int)(((float)k + 0.5f) * sv.inv_cap);
            const int slot = k - sp * sv.cap;
            const Real4 a = sv.atoms[(int)st[sp] * sv.cap + slot];
            const Real r2 = dist2(b, px, py, pz, a);
            core |= r2 < pp.hc2;
            acc_p += lj(r2, pp);
            if (TWO) acc_q += lj(dist2(b, qx, qy, qz, a), pp);
        }
    }
}

__global__ void __launch_bounds__(kWave * kMaxWalkersPerBlock) SWEEP_KERNEL(SweepArgs a)
{
    extern __shared__ __align__(32) unsigned char smem[];
    const int wave = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    const int blk = blockIdx.x;
    const int cid = a.block_class[blk];
    const ClassDev &C = a.cls[cid];
    const int nw = a.block_nw[blk];

    Real4 *slab = reinterpret_cast<Real4 *>(smem);
    int16_t *stencil = reinterpret_cast<int16_t *>(smem + (size_t)a.max_slab_len * sizeof(Real4));
    size_t st_bytes = ((size_t)a.max_stencil * sizeof(int16_t) + 31) & ~(size_t)31;
    Real4 *gas = reinterpret_cast<Real4 *>(smem + (size_t)a.max_slab_len * sizeof(Real4) + st_bytes) +
                 (size_t)wave * a.gas_stride;

    // ---- class slab and stencil into LDS (shared by the block's walkers) ----
    const int slab_len = C.slab_len;
    for (int k = threadIdx.x; k < slab_len; k += blockDim.x) {
#if defined(REGC_FP64)
        const double *src = a.slab4 + 4 * (size_t)(C.slab_off + k);
#else
        const float *src = a.slab4f + 4 * (size_t)(C.slab_off + k);
#endif
        Real4 v;
        v.x = src[0]; v.y = src[1]; v.z = src[2]; v.w = 0;
        slab[k] = v;
    }
    const int n_st = C.bins ? C.ncx * C.ncy * 9 : 0;
    for (int k = threadIdx.x; k < n_st; k += blockDim.x) stencil[k] = a.stencil[C.stencil_off + k];
    __syncthreads();
    if (wave >= nw) return;

    const int w = a.block_w0[blk] + wave;
    const int n_max = C.n_max;
    const int K = C.trials;

    // ---- walker state into LDS / registers ----
    int n = a.n[w];
    double e = a.e[w];
    const int label = a.label[w];
    const int sg = C.state_off + label;
    const double beta = a.beta[sg];
    const double lnz = a.lnz[sg];
    const double lnzv = lnz + C.lnv;
    {
        const double *src = a.xyz + (size_t)w * a.xyz_stride * 3;
        for (int k = lane; k < n; k += kWave) {
            Real4 v;
            v.x = (Real)src[3 * k]; v.y = (Real)src[3 * k + 1]; v.z = (Real)src[3 * k + 2]; v.w = 0;
            gas[k] = v;
        }
    }
    wave_sync();

    Box b;
    b.lx = (Real)C.lx; b.ly = (Real)C.ly; b.hx = (Real)C.half_lx; b.hy = (Real)C.half_ly;
    b.ix = (Real)C.inv_lx; b.iy = (Real)C.inv_ly;
    Pair gg, gs;
    gg.sig2 = (Real)a.pot.sig2_gg; gg.eps4 = (Real)a.pot.eps4_gg; gg.shift = (Real)a.pot.shift_gg;
    gg.rc2 = (Real)a.pot.rc2; gg.hc2 = (Real)a.pot.hc2_gg;
    gs.sig2 = (Real)a.pot.sig2_gs; gs.eps4 = (Real)a.pot.eps4_gs; gs.shift = (Real)a.pot.shift_gs;
    gs.rc2 = (Real)a.pot.rc2; gs.hc2 = (Real)a.pot.hc2_gs;
    const bool ideal = a.pot.ideal != 0;
    SlabView sv;
    sv.atoms = slab; sv.stencil = stencil; sv.len = slab_len; sv.bins = C.bins;
    sv.ncx = C.ncx; sv.ncy = C.ncy; sv.cap = C.cap; sv.inv_cap = C.bins ? 1.0f / (float)C.cap : 0.f;
    sv.inv_cw_x = (Real)C.inv_cw_x; sv.inv_cw_y = (Real)C.inv_cw_y;
    sv.top_plus_rc = (Real)(C.slab_top + sqrt(a.pot.rc2));
    const double lx = C.lx, ly = C.ly, zlo = C.zlo, zhi = C.zhi, H = C.zhi - C.zlo;
    const double md = a.max_disp;

    uint32_t st_cnt[kNStat];
#pragma unroll
    for (int k = 0; k < kNStat; ++k) st_cnt[k] = 0;

    for (int it = 0; it < a.n_sweeps; ++it) {
        const int64_t sweep = a.sweep0 + it;
        const bool tracing = a.trace_bits != nullptr && (sweep - a.trace_sweep0) < a.trace_cap &&
                             sweep >= a.trace_sweep0;
        for (int t0 = 0; t0 < K; t0 += 32) {
            // lane-parallel Philox: lane 2j -> block A of trial t0+j, lane 2j+1 -> block B
            const uint4 R = philox4x32_10(
                make_uint4((uint32_t)(t0 + (lane >> 1)), (uint32_t)sweep, (uint32_t)w, (uint32_t)(lane & 1)),
                a.key0, a.key1);
            const int tn = K - t0 < 32 ? K - t0 : 32;
            uint32_t bits = 0;
            for (int tt = 0; tt < tn; ++tt) {
                const uint32_t A0 = bcast(R.x, 2 * tt), A1 = bcast(R.y, 2 * tt);
                const uint32_t A2 = bcast(R.z, 2 * tt), A3 = bcast(R.w, 2 * tt);
                const uint32_t B0 = bcast(R.x, 2 * tt + 1), B1 = bcast(R.y, 2 * tt + 1);
                const uint32_t B2 = bcast(R.z, 2 * tt + 1);
                const double U = uniform53(B1, B2);
                bool accepted = false;
                if ((uint64_t)A0 < a.th_disp) {
                    // ---------------- displacement ----------------
                    st_cnt[0]++;
                    if (n == 0) {
                        st_cnt[7]++;
                    } else {
                        const int i = (int)(((uint64_t)A1 * (uint64_t)n) >> 32);
                        const Real4 o = gas[i];
                        double px = (double)o.x + md * (2.0 * uniform_open(A2) - 1.0);
                        double py = (double)o.y + md * (2.0 * uniform_open(A3) - 1.0);
                        const double pz = (double)o.z + md * (2.0 * uniform_open(B0) - 1.0);
                        if (px < 0.0) px += lx; else if (px >= lx) px -= lx;
                        if (py < 0.0) py += ly; else if (py >= ly) py -= ly;
                        if (pz < zlo || pz > zhi) {
                            st_cnt[8]++;
                        } else {
                            const Real qx = (Real)px, qy = (Real)py, qz = (Real)pz;
                            double de = 0.0;
                            bool core = false;
                            if (!ideal) {
                                Real en = 0, eo = 0;
                                for (int j = lane; j < n; j += kWave) {
                                    if (j == i) continue;
                                    const Real4 g = gas[j];
                                    const Real r2n = dist2(b, qx, qy, qz, g);
                                    core |= r2n < gg.hc2;
                                    en += lj(r2n, gg);
                                    eo += lj(dist2(b, o.x, o.y, o.z, g), gg);
                                }
                                const Real zmin = qz < o.z ? qz : o.z;
                                if (zmin < sv.top_plus_rc)
                                    slab_terms<true>(sv, b, gs, lane, qx, qy, qz, o.x, o.y, o.z, o.x, o.y, en, eo,
                                                     core);
#if defined(REGC_FP64)
                                const double sn = wave_sum(en), so = wave_sum(eo);
                                de = sn - so;
#else
                                de = (double)wave_sum(en - eo);
#endif
                                core = __any(core);
                            }
                            if (core) {
                                st_cnt[9]++;
                            } else {
                                accepted = metropolis(-beta * de, U);
                                if (accepted) {
                                    if (lane == 0) {
                                        Real4 v; v.x = qx; v.y = qy; v.z = qz; v.w = 0;
                                        gas[i] = v;
                                    }
                                    e += de;
                                    st_cnt[1]++;
                                }
                            }
                        }
                    }
                } else if ((uint64_t)A0 < a.th_ins) {
                    // ---------------- insertion ----------------
                    st_cnt[2]++;
                    if (n >= n_max) {
                        st_cnt[6]++;
                    } else {
                        const Real qx = (Real)(lx * uniform_open(A2));
                        const Real qy = (Real)(ly * uniform_open(A3));
                        const Real qz = (Real)(zlo + H * uniform_open(B0));
                        double de = 0.0;
                        bool core = false;
                        if (!ideal) {
                            Real en = 0, dummy = 0;
                            for (int j = lane; j < n; j += kWave) {
                                const Real r2 = dist2(b, qx, qy, qz, gas[j]);
                                core |= r2 < gg.hc2;
                                en += lj(r2, gg);
                            }
                            if (qz < sv.top_plus_rc)
                                slab_terms<false>(sv, b, gs, lane, qx, qy, qz, qx, qy, qz, qx, qy, en, dummy, core);
                            de = (double)wave_sum(en);
                            core = __any(core);
                        }
                        if (core) {
                            st_cnt[9]++;
                        } else {
                            accepted = metropolis((lnzv - a.lnk[n + 1]) - beta * de, U);
                            if (accepted) {
                                if (lane == 0) {
                                    Real4 v; v.x = qx; v.y = qy; v.z = qz; v.w = 0;
                                    gas[n] = v;
                                }
                                n += 1;
                                e += de;
                                st_cnt[3]++;
                            }
                        }
                    }
                } else {
                    // ---------------- removal ----------------
                    st_cnt[4]++;
                    if (n == 0) {
                        st_cnt[7]++;
                    } else {
                        const int i = (int)(((uint64_t)A1 * (uint64_t)n) >> 32);
                        const Real4 o = gas[i];
                        double de = 0.0;
                        if (!ideal) {
                            Real eo = 0, dummy = 0;
                            bool core = false;
                            for (int j = lane; j < n; j += kWave) {
                                if (j == i) continue;
                                eo += lj(dist2(b, o.x, o.y, o.z, gas[j]), gg);
                            }
                            if (o.z < sv.top_plus_rc)
                                slab_terms<false>(sv, b, gs, lane, o.x, o.y, o.z, o.x, o.y, o.z, o.x, o.y, eo, dummy,
                                                  core);
                            de = -(double)wave_sum(eo);
                        }
                        accepted = metropolis((a.lnk[n] - lnzv) - beta * de, U);
                        if (accepted) {
                            if (lane == 0 && i != n - 1) gas[i] = gas[n - 1];
                            n -= 1;
                            e += de;
                            st_cnt[5]++;
                        }
                    }
                }
                if (accepted) {
                    bits |= 1u << tt;
                    wave_sync();
                }
            }
            if (tracing && lane == 0)
                a.trace_bits[((size_t)(sweep - a.trace_sweep0) * a.n_walkers + w) * a.trace_words + (t0 >> 5)] = bits;
        }
        // ---- end of sweep: trace N, sample record ----
        if (lane == 0) {
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

    // ---- write back ----
    {
        double *dst = a.xyz + (size_t)w * a.xyz_stride * 3;
        for (int k = lane; k < n; k += kWave) {
            const Real4 v = gas[k];
            dst[3 * k] = (double)v.x; dst[3 * k + 1] = (double)v.y; dst[3 * k + 2] = (double)v.z;
        }
    }
    if (lane == 0) {
        a.n[w] = n;
        a.e[w] = e;
#pragma unroll
        for (int k = 0; k < kNStat; ++k)
            if (st_cnt[k]) atomicAdd(a.stats + (size_t)sg * kNStat + k, (unsigned long long)st_cnt[k]);
    }
}

// Full recomputation of each walker's energy (gas-gas pairs once, gas-slab for
// every atom), pair terms in Real, sums in FP64.  One wavefront per walker.
__global__ void __launch_bounds__(256) ENERGY_KERNEL(EnergyArgs a)
{
    const int w = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    if (w >= a.n_walkers) return;
    const ClassDev &C = a.cls[a.walker_class[w]];
    const int cid = a.walker_class[w];
    Box b;
    b.lx = (Real)C.lx; b.ly = (Real)C.ly; b.hx = (Real)C.half_lx; b.hy = (Real)C.half_ly;
    b.ix = (Real)C.inv_lx; b.iy = (Real)C.inv_ly;
    Pair gg, gs;
    gg.sig2 = (Real)a.pot.sig2_gg; gg.eps4 = (Real)a.pot.eps4_gg; gg.shift = (Real)a.pot.shift_gg;
    gg.rc2 = (Real)a.pot.rc2; gg.hc2 = (Real)a.pot.hc2_gg;
    gs.sig2 = (Real)a.pot.sig2_gs; gs.eps4 = (Real)a.pot.eps4_gs; gs.shift = (Real)a.pot.shift_gs;
    gs.rc2 = (Real)a.pot.rc2; gs.hc2 = (Real)a.pot.hc2_gs;
    const int n = a.n[w];
    const double *x = a.xyz + (size_t)w * a.xyz_stride * 3;
    const double *sl = a.slab4 + 4 * (size_t)a.unb_off[cid];
    const int ns = a.unb_len[cid];
    double acc = 0.0;
    if (!a.pot.ideal) {
        for (int i = 0; i < n; ++i) {
            const Real px = (Real)x[3 * i], py = (Real)x[3 * i + 1], pz = (Real)x[3 * i + 2];
            for (int j = i + 1 + lane; j < n; j += kWave) {
                Real4 q; q.x = (Real)x[3 * j]; q.y = (Real)x[3 * j + 1]; q.z = (Real)x[3 * j + 2]; q.w = 0;
                acc += (double)lj(dist2(b, px, py, pz, q), gg);
            }
            for (int k = lane; k < ns; k += kWave) {
                Real4 q; q.x = (Real)sl[4 * k]; q.y = (Real)sl[4 * k + 1]; q.z = (Real)sl[4 * k + 2]; q.w = 0;
                acc += (double)lj(dist2(b, px, py, pz, q), gs);
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) a.e_out[w] = acc;
}

hipError_t ENERGY_LAUNCH(const EnergyArgs &a, hipStream_t s)
{
    const int per = 4;
    hipLaunchKernelGGL(ENERGY_KERNEL, dim3((a.n_walkers + per - 1) / per), dim3(kWave * per), 0, s, a);
    return hipGetLastError();
}

hipError_t SWEEP_LAUNCH(const SweepArgs &a, int n_blocks, int wpb, size_t smem, hipStream_t s)
{
    hipLaunchKernelGGL(SWEEP_KERNEL, dim3(n_blocks), dim3(kWave * wpb), smem, s, a);
    return hipGetLastError();
}

}  // namespace regc
