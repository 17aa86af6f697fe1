// sweep.hip -- the REGC sweep kernel: K grand-canonical / displacement trials per
// sweep for every walker, its gas coordinates and its class's frozen slab resident
// in LDS for the whole launch; plus the full energy recomputation kernel.
//
// This file is compiled twice:
//   -DREGC_FP64 with -ffp-contract=off : every operation in FP64 (trajectory-parity
//                                        mode: the same decisions as a sequential FP64
//                                        evaluation up to summation order and the last
//                                        bit of log);
//   -DREGC_FP32                        : pair terms and their per-lane sums in FP32;
//                                        running energy and acceptance test in FP64.
//
// Per trial (arXiv:1908.11118, Sec. II.A.1 and II.A.3):
//   move type from word A0 (displacement / insertion / removal, thresholds set
//   from p_disp, p_ins); the affected particle i = floor(A1 * N / 2^32);
//   displacement by a uniform vector in the cube [-d, d]^3, Eq. (7): ln A = -beta dE;
//   insertion at a uniform point of V, Eq. (3) with the exponent read as
//   beta [mu - (E_{N+1} - E_N)]: ln A = ln z + ln V - ln(N+1) - beta dE;
//   removal, Eq. (2): ln A = ln N - ln z - ln V - beta dE;
//   accept when U53 <= min(1, A), evaluated as dE <= (ln prefactor - ln U) / beta.
// dE sums LJ pair terms of the moved particle over the other gas atoms and over
// the slab atoms (all of them, or those of the 3x3 block of x-y columns around
// the particle).  Storage rule: insertion appends, removal moves the last particle
// into the freed slot.
//
// Launch variants (template parameters):
//   SPLIT = 1: one wavefront per walker, several walkers per workgroup;
//   SPLIT = 2, 4: one walker per workgroup of SPLIT wavefronts; each takes every
//              SPLIT-th block of candidates, the partial sums meet in LDS behind a
//              barrier (added in wave order), every wave then takes the same decision
//              and writes an accepted update into the walker's LDS copy.  Several
//              waves per SIMD hide latency when walkers are as few as SIMDs.
//   CULL  = false: every candidate pair is evaluated in full;
//   CULL  = true : a first pass computes squared distances only and queues the pairs
//              inside the cutoff in LDS (compacted across the wave); the LJ terms are
//              evaluated on the queue only.
#include "sweep_dev.h"
#include "swap_dev.h"

#if defined(REGC_FP64)
#define SWEEP_LAUNCH launch_sweep_f64
#define PERSIST_LAUNCH launch_sweep_persist_f64
#define PERSIST_CAPACITY persist_capacity_f64
#define PAPER_LAUNCH launch_paper_f64
#define ENERGY_KERNEL energy_kernel_f64
#define ENERGY_LAUNCH launch_energy_f64
#else
#define SWEEP_LAUNCH launch_sweep_f32
#define PERSIST_LAUNCH launch_sweep_persist_f32
#define PERSIST_CAPACITY persist_capacity_f32
#define PAPER_LAUNCH launch_paper_f32
#define ENERGY_KERNEL energy_kernel_f32
#define ENERGY_LAUNCH launch_energy_f32
#endif

namespace regc {
namespace REGC_PREC {

// Waves per SIMD the one-trial kernel's register budget must allow: four in the FP32
// build with one wave per walker (128 VGPRs, no spills), so that four walkers share
// each SIMD (measured 2.03e9 against 1.60e9 trial moves/s at 4096 walkers on 256 CUs),
// and with four waves per walker (128 VGPRs and a few spilled bytes: 1024 walkers are
// 4096 waves, which fit at once only at four per SIMD; 3.10 against 4.46 ms per
// launch); with two waves per walker, and in the FP64 build, the registers stay as
// they are (a 128-register budget spills there and was measured slower).
#if defined(REGC_FP64)
constexpr int kSweepWavesPerSimd = 1;
#else
constexpr int kSweepWavesPerSimd = 4;
#endif

// Grid-wide barrier of the persistent launch (every workgroup resident: cooperative
// launch).  Thread 0 of each workgroup arrives on gbar[0]; the last to arrive resets it
// and advances the generation gbar[1], which the others wait for.  A wait is bounded:
// past the bound the workgroup sets gerr and goes on, so the launch always ends (the
// host then reports the run as failed).
constexpr unsigned kGridSpinLimit = 1u << 26;

__device__ __forceinline__ void grid_sync(const SweepArgs &a)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned *bar = a.gbar;
        const unsigned gen = __hip_atomic_load(bar + 1, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        const unsigned arrived = __hip_atomic_fetch_add(bar, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == gridDim.x - 1) {
            __hip_atomic_store(bar, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(bar + 1, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            unsigned spins = 0;
            while (__hip_atomic_load(bar + 1, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                __builtin_amdgcn_s_sleep(2);
                if (++spins == kGridSpinLimit) {
                    atomicOr(a.gerr, 1);
                    break;
                }
            }
        }
        __threadfence();
    }
    __syncthreads();
}

// The one-trial sweep (template body of sweep_kernel and sweep_persist_kernel).
// PERSIST: whole exchange intervals in one launch; after every swap_every-th sweep
// each walker publishes N and E, the workgroups meet at a grid barrier, workgroup c
// (wave 0) runs the exchange step of class c, they meet again, and every walker
// reads its new state.
template <int SPLIT, bool CULL, bool PERSIST>
__device__ __forceinline__ void sweep_body(const SweepArgs &a)
{
    extern __shared__ __align__(32) unsigned char smem[];
    const int wave = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    const int slot = wave / SPLIT;              // walker within the block
    const int part = wave % SPLIT;              // this wave's share of the candidates
    const int waves = blockDim.x / kWave;
    const int blk = blockIdx.x;
    const int cid = a.block_class[blk];
    const ClassDev &C = a.cls[cid];
    const int nw = a.block_nw[blk];

    const LdsLayout L = lds_layout(a.max_slab_len, a.gas_stride, a.max_slab_scan, waves / SPLIT,
                                   CULL ? waves : 0, (int)sizeof(Real));
    Real4 *slab = reinterpret_cast<Real4 *>(smem + L.slab);
    double *lnk = reinterpret_cast<double *>(smem + L.lnk);
    double *xch = reinterpret_cast<double *>(smem + L.xch) + slot * 16;    // [parity][part][value, core]
    Real4 *gas = reinterpret_cast<Real4 *>(smem + L.gas) + (size_t)slot * a.gas_stride;
    Real *qgas = reinterpret_cast<Real *>(smem + L.queue) + (size_t)wave * (2 * a.gas_stride + 2 * a.max_slab_scan);
    Real *qslab = qgas + 2 * a.gas_stride;

    // ---- class slab and log table into LDS (shared by the block) ----
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
    for (int k = threadIdx.x; k < a.gas_stride + 2; k += blockDim.x) lnk[k] = a.lnk[k];
    __syncthreads();
    if (slot >= nw) {          // (blocks with SPLIT > 1 always hold one walker)
        if (PERSIST)           // a wave without a walker still meets every grid barrier
            for (int k = 0; k < a.n_sweeps / a.swap_every; ++k) {
                grid_sync(a);
                grid_sync(a);
            }
        return;
    }

    const int w = a.wslot ? a.wslot[a.block_w0[blk] + slot] : a.block_w0[blk] + slot;
    const int n_max = C.n_max;
    const int K = C.trials;

    // ---- walker state into LDS / registers ----
    int n = a.n[w];
    if (SPLIT == 1 && a.wslot) {
        // one wave per walker and several walkers per SIMD (the walker order by cost is
        // on): the more atoms the walker holds relative to its class's cap, the higher its
        // wave's issue priority, so that the longest chains of trials, which end the
        // launch, do not wait behind shorter ones (config 3: 10.89 -> 10.08 ms per launch;
        // 4096 walkers of config 2's system: 3.57 -> 3.41 ms).  With two waves per walker
        // the same rule made config 2 2.3 % slower, so it stays with one.
        const int pn = (4 * __builtin_amdgcn_readfirstlane(n)) / (C.n_max + 1);
        if (pn >= 3) __builtin_amdgcn_s_setprio(3);
        else if (pn == 2) __builtin_amdgcn_s_setprio(2);
        else if (pn == 1) __builtin_amdgcn_s_setprio(1);
    }
    double e = a.e[w];
    int label = a.label[w];
    int sg = C.state_off + label;
    double beta = a.beta[sg];
    double lnz = a.lnz[sg];
    double lnzv = in_vgpr(lnz + C.lnv);
    {
        const double *src = a.xyz + (size_t)w * a.xyz_stride * 3;
        for (int k = part * kWave + lane; k < n; k += SPLIT * kWave) {
            Real4 v;
            v.x = (Real)src[3 * k]; v.y = (Real)src[3 * k + 1]; v.z = (Real)src[3 * k + 2]; v.w = 0;
            gas[k] = v;
        }
    }
    if (SPLIT == 1) wave_sync(); else __syncthreads();

    Box b;
    b.lx = in_vgpr((Real)C.lx); b.ly = in_vgpr((Real)C.ly);
    b.hx = in_vgpr((Real)C.half_lx); b.hy = in_vgpr((Real)C.half_ly);
    b.ix = in_vgpr((Real)C.inv_lx); b.iy = in_vgpr((Real)C.inv_ly);
    Pair gg, gs;
    gg.sig2 = in_vgpr((Real)a.pot.sig2_gg); gg.eps4 = in_vgpr((Real)a.pot.eps4_gg);
    gg.shift = in_vgpr((Real)a.pot.shift_gg); gg.rc2 = in_vgpr((Real)a.pot.rc2); gg.hc2 = in_vgpr((Real)a.pot.hc2_gg);
    gs.sig2 = in_vgpr((Real)a.pot.sig2_gs); gs.eps4 = in_vgpr((Real)a.pot.eps4_gs);
    gs.shift = in_vgpr((Real)a.pot.shift_gs); gs.rc2 = gg.rc2; gs.hc2 = in_vgpr((Real)a.pot.hc2_gs);
    const bool ideal = a.pot.ideal != 0;
    SlabView sv;
    sv.atoms = slab; sv.len = slab_len; sv.bins = C.bins;
    sv.ncx = C.ncx; sv.ncy = C.ncy; sv.cap = C.cap;
    sv.inv_cap = in_vgpr(C.bins ? 1.0f / (float)C.cap : 0.f);
    sv.inv_cw_x = in_vgpr((Real)C.inv_cw_x); sv.inv_cw_y = in_vgpr((Real)C.inv_cw_y);
    sv.top_plus_rc = in_vgpr((Real)(C.slab_top + sqrt(a.pot.rc2)));
    // The proposal is computed in the pair terms' precision: FP64 in the FP64 build
    // (the oracle's arithmetic, below), FP32 with FP32 pair terms -- one broadcast per
    // uniform instead of two and FP32 instead of FP64 operations on the trial's chain
    // (config 2: 2.51 -> 2.43 ms per launch).  The acceptance test is FP64 in both.
    // The FP64 constants are declared in both builds: the FP32 build measured 1.5 %
    // faster with them present than without (register allocation of the trial loop).
    const double lx = in_vgpr(C.lx), ly = in_vgpr(C.ly), zlo = in_vgpr(C.zlo), zhi = in_vgpr(C.zhi);
    const double H = in_vgpr(C.zhi - C.zlo);
    const double md = in_vgpr(a.max_disp);
    double tinv = in_vgpr(1.0 / beta);
#if !defined(REGC_FP64)
    const float mdf = in_vgpr((float)a.max_disp), zlof = in_vgpr((float)C.zlo), zhif = in_vgpr((float)C.zhi);
    const float Hf = in_vgpr((float)(C.zhi - C.zlo));
#endif
    const int slab_scan = C.bins ? 9 * C.cap : slab_len;

    uint32_t stat = 0;     // lane k < kNStat holds counter k
    uint32_t useful = 0;   // per lane: evaluated pairs inside the cutoff
    uint64_t cand = 0;     // wave-uniform: candidate pairs of all parts
    uint32_t xcount = 0;   // exchanges so far: consecutive exchanges use alternate slots

    const int64_t sweep_first = a.clock ? a.clock[0] + a.sweep0 : a.sweep0;
    for (int it = 0; it < a.n_sweeps; ++it) {
        const int64_t sweep = sweep_first + it;
        const bool tracing = a.trace_bits != nullptr && (sweep - a.trace_sweep0) < a.trace_cap &&
                             sweep >= a.trace_sweep0;
        for (int t0 = 0; t0 < K; t0 += 32) {
            // (several waves per walker: the batch's random numbers, bulk vector work, at
            // the lowest issue priority like the pair loop; config 2: 2.39 -> 2.36 ms)
            if (SPLIT >= 2) __builtin_amdgcn_s_setprio(0);
            // lane-parallel Philox: lane 2j -> block A of trial t0+j, lane 2j+1 -> block B
            const uint4 R = philox4x32_10(
                make_uint4((uint32_t)(t0 + (lane >> 1)), (uint32_t)sweep, (uint32_t)w, (uint32_t)(lane & 1)),
                a.key0, a.key1);
            // FP64 uniforms of the batch, lane-parallel: on A lanes f0, f1 are the x, y
            // uniforms (A2, A3); on B lanes f2 is the z uniform (B0) and f3 = ln U (B1, B2).
            const double f0 = uniform_open(R.z), f1 = uniform_open(R.w), f2 = uniform_open(R.x);
            const double f3 = log(uniform53(R.y, R.z));
#if !defined(REGC_FP64)
            const float g0 = (float)f0, g1 = (float)f1, g2 = (float)f2;     // FP32 build: x, y, z uniforms
#endif
            const int tn = K - t0 < 32 ? K - t0 : 32;
            if (SPLIT >= 2) __builtin_amdgcn_s_setprio(2);
            uint32_t bits = 0;
            for (int tt = 0; tt < tn; ++tt) {
                const uint32_t A0 = bcast(R.x, 2 * tt), A1 = bcast(R.y, 2 * tt);
                // one wave per walker: the first step's gas atoms are read at the top of the
                // trial, their LDS round trip overlapping the proposal (4 % faster with one
                // wave per walker at 1024 walkers, 2 % at 4096)
                Real4 pre[2];
                if (SPLIT == 1) {
                    pre[0] = gas[lane < n ? lane : 0];
                    pre[1] = gas[lane + kWave < n ? lane + kWave : 0];
                }
                // move type: 0 displacement, 1 insertion, 2 removal
                const int kind = (uint64_t)A0 < a.th_disp ? 0 : ((uint64_t)A0 < a.th_ins ? 1 : 2);
                stat += lane == 2 * kind;
                bool accepted = false;
                if (kind == 1 ? n >= n_max : n == 0) {
                    stat += lane == (kind == 1 ? 6 : 7);          // cap / empty
                } else {
                    const double lnU = bcast(f3, 2 * tt + 1);
#if defined(REGC_FP64)
                    const double ux = bcast(f0, 2 * tt), uy = bcast(f1, 2 * tt), uz = bcast(f2, 2 * tt + 1);
                    const int i = kind == 1 ? -1 : (int)(((uint64_t)A1 * (uint64_t)n) >> 32);
                    const Real4 o = gas[kind == 1 ? 0 : i];
                    // two waves per walker: the last particle too (moved into slot i by
                    // an accepted removal), read together with particle i, off the chain
                    // of an accepted move
                    Real4 last = o;
                    if (SPLIT == 2) last = gas[n > 0 ? n - 1 : 0];
                    double px = 0.0, py = 0.0, pz = 0.0, c;
                    bool wall = false;
                    if (kind == 0) {
                        px = (double)o.x + md * (2.0 * ux - 1.0);
                        py = (double)o.y + md * (2.0 * uy - 1.0);
                        pz = (double)o.z + md * (2.0 * uz - 1.0);
                        if (px < 0.0) px += lx; else if (px >= lx) px -= lx;
                        if (py < 0.0) py += ly; else if (py >= ly) py -= ly;
                        wall = pz < zlo || pz > zhi;
                        c = 0.0;
                    } else if (kind == 1) {
                        px = lx * ux;
                        py = ly * uy;
                        pz = zlo + H * uz;
                        c = lnzv - lnk[n + 1];                    // ln z V / (N+1)
                    } else {
                        c = lnk[n] - lnzv;                        // ln N / (z V)
                    }
#else
                    // the same trial in FP32 (particle, last particle and prefactors as above)
                    const float ux = bcast(g0, 2 * tt), uy = bcast(g1, 2 * tt), uz = bcast(g2, 2 * tt + 1);
                    const int i = kind == 1 ? -1 : (int)(((uint64_t)A1 * (uint64_t)n) >> 32);
                    const Real4 o = gas[kind == 1 ? 0 : i];
                    Real4 last = o;
                    if (SPLIT == 2) last = gas[n > 0 ? n - 1 : 0];
                    float px = 0.f, py = 0.f, pz = 0.f;
                    double c;
                    bool wall = false;
                    if (kind == 0) {
                        px = o.x + mdf * (2.f * ux - 1.f);
                        py = o.y + mdf * (2.f * uy - 1.f);
                        pz = o.z + mdf * (2.f * uz - 1.f);
                        if (px < 0.f) px += b.lx; else if (px >= b.lx) px -= b.lx;
                        if (py < 0.f) py += b.ly; else if (py >= b.ly) py -= b.ly;
                        wall = pz < zlof || pz > zhif;
                        c = 0.0;
                    } else if (kind == 1) {
                        px = b.lx * ux;
                        py = b.ly * uy;
                        pz = zlof + Hf * uz;
                        c = lnzv - lnk[n + 1];
                    } else {
                        c = lnk[n] - lnzv;
                    }
#endif
                    if (wall) {
                        stat += lane == 8;
                    } else {
                        // accept iff ln U <= ln prefactor - beta dE (U <= min(1, A))
                        const double thr = (c - lnU) * tinv;
                        const Real qx = (Real)px, qy = (Real)py, qz = (Real)pz;
                        double de = 0.0;
                        bool core = false;
                        if (!ideal) {
                            Real pd;
                            // two waves per walker: the pair loop at the lowest issue priority,
                            // the rest of the trial (the reduction, the exchange between the
                            // waves, the decision, the update and the next proposal) at a higher
                            // one, so that where two walkers share a SIMD the one on its serial
                            // path issues first (config 2: 2.43 -> 2.38 ms per launch; four waves
                            // per walker: 2.93 -> 2.71 ms)
                            if (SPLIT >= 2) __builtin_amdgcn_s_setprio(0);
                            if (kind == 0)
                                pd = partial_delta<true, true, SPLIT, CULL, SPLIT == 1>(gas, n, i, sv, b, gg, gs, lane, part, qx,
                                                                            qy, qz, o.x, o.y, o.z, qgas, qslab, core,
                                                                            useful, pre);
                            else if (kind == 1)
                                pd = partial_delta<true, false, SPLIT, CULL, SPLIT == 1>(gas, n, -1, sv, b, gg, gs, lane, part,
                                                                             qx, qy, qz, qx, qy, qz, qgas, qslab,
                                                                             core, useful, pre);
                            else
                                pd = partial_delta<false, true, SPLIT, CULL, SPLIT == 1>(gas, n, i, sv, b, gg, gs, lane, part,
                                                                             o.x, o.y, o.z, o.x, o.y, o.z, qgas,
                                                                             qslab, core, useful, pre);
                            if (SPLIT == 4) __builtin_amdgcn_s_setprio(2);   // (two waves: from the reduction on)
                            if (SPLIT == 1) {
                                de = (double)pd;
                            } else {
                                // alternate slots: exchange k+2 reuses the slot of exchange k
                                // only after every wave passed the barrier of exchange k+1
                                double *mine = xch + ((xcount & 1) * SPLIT + part) * 2;
                                if (lane == 0) {
                                    mine[0] = (double)pd;
                                    mine[1] = core ? 1.0 : 0.0;
                                }
                                __syncthreads();
                                const double *x0 = xch + (xcount & 1) * SPLIT * 2;
                                de = x0[0];
                                double cf = x0[1];
#pragma unroll
                                for (int q = 1; q < SPLIT; ++q) {
                                    de += x0[2 * q];
                                    cf += x0[2 * q + 1];
                                }
                                core = cf != 0.0;
                                ++xcount;
                            }
                            const uint64_t mult = kind == 0 ? 2 : 1;
                            const Real zmin = kind == 0 ? (qz < o.z ? qz : o.z) : (kind == 1 ? qz : o.z);
                            cand += mult * (uint64_t)((kind == 1 ? n : n - 1) +
                                                      (zmin < sv.top_plus_rc ? slab_scan : 0));
                        }
                        if (core && kind != 2) {
                            stat += lane == 9;
                        } else if (de <= thr) {
                            accepted = true;
                            stat += lane == 2 * kind + 1;
                            e += de;
                            // every wave of the walker writes the update into the shared
                            // LDS copy itself (the same value), so a wave needs only its own
                            // write to be visible.  Across waves, the exchange barrier of
                            // this trial ordered all reads before these writes, and that of
                            // the next trial orders these writes before any later one.  The
                            // ideal gas has no exchange: its barrier here keeps the other
                            // wave's read of this trial's particle before the writes, and the
                            // one below keeps the writes before the next trial's reads.
                            if (SPLIT > 1 && ideal) __syncthreads();
                            if (SPLIT == 2) {
                                // one store for every move type: the new position into slot
                                // i (displacement) or n (insertion), the last particle into
                                // slot i (removal; the same value again when i is the last).
                                // Measured 1.4 % faster with two waves per walker at 1024
                                // walkers, 2-3 % slower with one (hence the two forms).
                                Real4 v;
                                v.x = kind == 2 ? last.x : qx;
                                v.y = kind == 2 ? last.y : qy;
                                v.z = kind == 2 ? last.z : qz;
                                v.w = 0;
                                if (lane == 0) gas[kind == 1 ? n : i] = v;
                                n += kind == 1 ? 1 : (kind == 2 ? -1 : 0);
                            } else if (kind == 0) {
                                if (lane == 0) {
                                    Real4 v; v.x = qx; v.y = qy; v.z = qz; v.w = 0;
                                    gas[i] = v;
                                }
                            } else if (kind == 1) {
                                if (lane == 0) {
                                    Real4 v; v.x = qx; v.y = qy; v.z = qz; v.w = 0;
                                    gas[n] = v;
                                }
                                n += 1;
                            } else {
                                if (lane == 0 && i != n - 1) gas[i] = gas[n - 1];
                                n -= 1;
                            }
                        }
                    }
                }
                if (accepted) {
                    bits |= 1u << tt;
                    if (SPLIT == 1 || !ideal) wave_sync(); else __syncthreads();
                }
            }
            if (tracing && part == 0 && lane == 0)
                a.trace_bits[((size_t)(sweep - a.trace_sweep0) * a.n_walkers + w) * a.trace_words + (t0 >> 5)] = bits;
        }
        // ---- end of sweep: running energy resynchronised, trace N, sample record ----
        if (a.resync_every > 0 && (sweep + 1) % a.resync_every == 0 && !ideal) {
            const double pe = full_energy_part<SPLIT>(gas, n, sv, b, gg, gs, lane, part);
            if (SPLIT == 1) {
                e = pe;
            } else {
                double *mine = xch + ((xcount & 1) * SPLIT + part) * 2;
                if (lane == 0) mine[0] = pe;
                __syncthreads();
                const double *x0 = xch + (xcount & 1) * SPLIT * 2;
                e = x0[0];
#pragma unroll
                for (int q = 1; q < SPLIT; ++q) e += x0[2 * q];
                ++xcount;
            }
        }
        if (part == 0 && lane == 0) {
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
        if (PERSIST && (sweep + 1) % a.swap_every == 0) {
            // ---- the exchange step inside the launch ----
            if (part == 0) {
                if (lane < kNStat && stat) atomicAdd(a.stats + (size_t)sg * kNStat + lane, (unsigned long long)stat);
                if (lane == 0) {
                    a.n[w] = n;
                    a.e[w] = e;
                }
                __threadfence();       // this wave's stores visible to every workgroup
            }
            stat = 0;
            grid_sync(a);
            if (blk < a.n_class && threadIdx.x < kWave) {
                swap_class<true>(a.sw, blk, (sweep + 1) / a.swap_every - 1, lane, kWave);
                __threadfence();
            }
            grid_sync(a);
            label = __hip_atomic_load(a.label + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            sg = C.state_off + label;
            beta = a.beta[sg];
            lnz = a.lnz[sg];
            lnzv = in_vgpr(lnz + C.lnv);
            tinv = in_vgpr(1.0 / beta);
        }
    }

    // ---- write back ----
    if (SPLIT > 1) __syncthreads();
    {
        double *dst = a.xyz + (size_t)w * a.xyz_stride * 3;
        for (int k = part * kWave + lane; k < n; k += SPLIT * kWave) {
            const Real4 v = gas[k];
            dst[3 * k] = (double)v.x; dst[3 * k + 1] = (double)v.y; dst[3 * k + 2] = (double)v.z;
        }
    }
    {
        uint32_t u = useful;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) u += __shfl_xor(u, o);
        if (lane == 0 && a.pairs) {
            if (part == 0) atomicAdd(a.pairs, (unsigned long long)cand);
            atomicAdd(a.pairs + 1, (unsigned long long)u);
        }
    }
    if (part == 0) {
        if (lane < kNStat && stat) atomicAdd(a.stats + (size_t)sg * kNStat + lane, (unsigned long long)stat);
        if (lane == 0) {
            a.n[w] = n;
            a.e[w] = e;
        }
    }
}

template <int SPLIT, bool CULL>
__global__ void __launch_bounds__(kWave * kMaxWalkersPerBlock, SPLIT != 2 ? kSweepWavesPerSimd : 1)
    sweep_kernel(SweepArgs a)
{
    sweep_body<SPLIT, CULL, false>(a);
}

template <int SPLIT>
__global__ void __launch_bounds__(kWave * kMaxWalkersPerBlock) sweep_persist_kernel(SweepArgs a)
{
    sweep_body<SPLIT, false, true>(a);
}

// ---- batched trials -------------------------------------------------------------
// The trials of one walker form a chain, and with one walker per SIMD a trial's
// dependent steps (broadcasts, LDS round trips, reductions, the decision) leave the
// vector unit idle.  This kernel evaluates B consecutive trials t .. t+B-1 of a walker
// at once, G = 64 / B lanes each, against the configuration X0 at the start of the
// batch, and then decides them in order, each exactly as the one-trial-at-a-time chain
// would:
//   - the energy change of trial h on the current configuration is its value on X0
//     plus, for every earlier trial g of the batch that was accepted, the pair terms
//     between h's positions and g's: with P the new position of a trial (displacement
//     target, insertion point) and Q the old one (displaced or removed particle),
//       dE_h += [phi(P_h - P_g) - phi(Q_h - P_g)] - [phi(P_h - Q_g) - phi(Q_h - Q_g)],
//     computed in the same pass (lane 4 g + k of h's group holds term k), and a new
//     pair P_h, P_g closer than the hard core rejects h;
//   - trial h is evaluated again in the next pass (the batch ends before it) when an
//     earlier accepted trial of the batch changed what h proposes or what its X0 value
//     assumed: its particle index floor(A1 N / 2^32) under the current N, its particle
//     (a slot whose occupant changed: displaced, refilled by a removal, emptied by a
//     removal, filled by an insertion), an insertion no longer at the cap or a
//     particle present in a walker that was empty, or a hard-core flag raised on X0;
//   - the Metropolis test uses the prefactor of the current N.
// Each particle's energy with the frozen slab is kept in LDS (computed at the start of
// the launch, replaced when the particle moves), so a displacement sums slab terms at
// its new position only and a removal none.  The accept/reject sequence, N, the
// coordinates and the counters are those of the sequential chain; energies differ
// only in the order of the sum.  Trial 0 of every batch is exact, so each pass decides
// at least one trial.  COUNT adds the count of pair terms inside the cutoff.
template <int B, bool COUNT>
__global__ void __launch_bounds__(kWave * kMaxWalkersPerBlock) batch_kernel(SweepArgs a)
{
    constexpr int G = kWave / B;
    static_assert(G >= 4 * (B - 1), "a group must hold the pair terms with all earlier trials");
    extern __shared__ __align__(32) unsigned char smem[];
    // the wave index is the same in all lanes; readfirstlane lets the compiler know, so
    // the walker index and the chain's state (N, E, the decisions) live in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x % kWave;
    const int grp = lane / G, gl = lane % G;
    const int waves = blockDim.x / kWave;
    const int blk = blockIdx.x;
    const int cid = a.block_class[blk];
    const ClassDev &C = a.cls[cid];
    const int nw = a.block_nw[blk];

    const BatchLds L = batch_lds(a.max_slab_len, a.gas_stride, waves, (int)sizeof(Real));
    Real4 *slab = reinterpret_cast<Real4 *>(smem + L.slab);
    double *lnk = reinterpret_cast<double *>(smem + L.lnk);
    Real4 *gas = reinterpret_cast<Real4 *>(smem + L.gas) + (size_t)wave * a.gas_stride;
    Real *eslab = reinterpret_cast<Real *>(smem + L.eslab) + (size_t)wave * a.gas_stride;

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
    for (int k = threadIdx.x; k < a.gas_stride + 2; k += blockDim.x) lnk[k] = a.lnk[k];
    __syncthreads();
    if (wave >= nw) return;

    const int w = a.block_w0[blk] + wave;
    const int n_max = C.n_max;
    const int K = C.trials;
    int n = a.n[w];
    double e = a.e[w];
    const int label = a.label[w];
    const int sg = C.state_off + label;
    const double beta = a.beta[sg];
    const double lnz = a.lnz[sg];
    const double lnzv = lnz + C.lnv;

    // wave-uniform constants kept in VGPRs: the loop holds more uniform values than
    // there are SGPRs, and spilled SGPRs cost a lane read per use
    Box b;
    b.lx = in_vgpr((Real)C.lx); b.ly = in_vgpr((Real)C.ly); b.hx = in_vgpr((Real)C.half_lx);
    b.hy = in_vgpr((Real)C.half_ly); b.ix = in_vgpr((Real)C.inv_lx); b.iy = in_vgpr((Real)C.inv_ly);
    Pair gg, gs;
    gg.sig2 = in_vgpr((Real)a.pot.sig2_gg); gg.eps4 = in_vgpr((Real)a.pot.eps4_gg);
    gg.shift = in_vgpr((Real)a.pot.shift_gg); gg.rc2 = in_vgpr((Real)a.pot.rc2); gg.hc2 = in_vgpr((Real)a.pot.hc2_gg);
    gs.sig2 = in_vgpr((Real)a.pot.sig2_gs); gs.eps4 = in_vgpr((Real)a.pot.eps4_gs);
    gs.shift = in_vgpr((Real)a.pot.shift_gs); gs.rc2 = gg.rc2; gs.hc2 = in_vgpr((Real)a.pot.hc2_gs);
    const bool ideal = a.pot.ideal != 0;
    SlabView sv;
    sv.atoms = slab; sv.len = slab_len; sv.bins = C.bins;
    sv.ncx = C.ncx; sv.ncy = C.ncy; sv.cap = C.cap;
    sv.inv_cap = in_vgpr(C.bins ? 1.0f / (float)C.cap : 0.f);
    sv.inv_cw_x = in_vgpr((Real)C.inv_cw_x); sv.inv_cw_y = in_vgpr((Real)C.inv_cw_y);
    sv.top_plus_rc = in_vgpr((Real)(C.slab_top + sqrt(a.pot.rc2)));
    const double lx = in_vgpr(C.lx), ly = in_vgpr(C.ly), zlo = in_vgpr(C.zlo), zhi = in_vgpr(C.zhi);
    const double H = in_vgpr(C.zhi - C.zlo);
    const double md = in_vgpr(a.max_disp);
    const double tinv = in_vgpr(1.0 / beta);
    const double lnzv_v = in_vgpr(lnzv);
    const int slab_scan = C.bins ? 9 * C.cap : slab_len;
    Real4 far;                      // a position beyond the cutoff of every atom: absent P or Q
    far.x = 0; far.y = 0; far.z = (Real)1.0e4; far.w = 0;

    // coordinates, and each particle's slab energy (lane per particle, slab entries in order)
    {
        const double *src = a.xyz + (size_t)w * a.xyz_stride * 3;
        for (int k = lane; k < n; k += kWave) {
            Real4 v;
            v.x = (Real)src[3 * k]; v.y = (Real)src[3 * k + 1]; v.z = (Real)src[3 * k + 2]; v.w = 0;
            gas[k] = v;
            Real es = 0;
            if (!ideal && v.z < sv.top_plus_rc) {
                int cx = 0, cy = 0;
                if (sv.bins) column_of_lanes(sv, v.x, v.y, cx, cy);
                for (int q = 0; q < slab_scan; ++q)
                    es += lj(dist2(b, v.x, v.y, v.z, sv.atoms[sv.bins ? block_entry(sv, cx, cy, q) : q]), gs);
            }
            eslab[k] = es;
        }
    }
    wave_sync();

    uint32_t stat = 0;     // lane k < kNStat holds counter k
    uint32_t useful = 0;
    uint64_t cand = 0;

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
            const int tn = K - t0 < 32 ? K - t0 : 32;
            uint32_t bits = 0;
            for (int t = 0; t < tn;) {
                const int nb = tn - t < B ? tn - t : B;
                const int n0 = n;
                const bool act = grp < nb;
                // this group's trial t + grp: words of Philox blocks A (lane 2m) and B (lane 2m + 1)
                const int src = 2 * (t + (act ? grp : 0));
                const uint32_t A0 = (uint32_t)__shfl((int)R.x, src);
                const uint32_t A1 = (uint32_t)__shfl((int)R.y, src);
                const double ux = __shfl(f0, src), uy = __shfl(f1, src);
                const double uz = __shfl(f2, src + 1), lnU = __shfl(f3, src + 1);
                const int kind = (uint64_t)A0 < a.th_disp ? 0 : ((uint64_t)A0 < a.th_ins ? 1 : 2);
                const bool skip = kind == 1 ? n0 >= n_max : n0 == 0;
                const int i = kind == 1 || skip ? 0 : (int)(((uint64_t)A1 * (uint64_t)n0) >> 32);
                const int ex = kind == 1 ? -1 : i;                // the gas atom left out of the sum
                const Real4 o = gas[i];
                const Real eo = kind == 1 || skip ? Real(0) : eslab[i];
                // (the kinds differ between the wave's groups: selects, not branches)
                double dx = (double)o.x + md * (2.0 * ux - 1.0);
                double dy = (double)o.y + md * (2.0 * uy - 1.0);
                const double dz = (double)o.z + md * (2.0 * uz - 1.0);
                dx = dx < 0.0 ? dx + lx : (dx >= lx ? dx - lx : dx);
                dy = dy < 0.0 ? dy + ly : (dy >= ly ? dy - ly : dy);
                const double px = kind == 0 ? dx : lx * ux;
                const double py = kind == 0 ? dy : ly * uy;
                const double pz = kind == 0 ? dz : zlo + H * uz;
                const bool wall = (kind == 0) & !skip & ((dz < zlo) | (dz > zhi));
                const double ln0 = lnk[n0], ln1 = lnk[n0 + 1];
                // 0, ln z V / (N+1) or ln N / (z V)
                const double c = kind == 0 ? 0.0 : (kind == 1 ? lnzv_v - ln1 : ln0 - lnzv_v);
                const double thr = (c - lnU) * tinv;              // accept iff dE <= thr
                const bool live = act && !skip && !wall;          // the trial moves a particle
                const bool compute = live && !ideal;
                Real4 P = far, Q = far;
                if (live && kind != 2) { P.x = (Real)px; P.y = (Real)py; P.z = (Real)pz; }
                if (live && kind != 1) { Q.x = o.x; Q.y = o.y; Q.z = o.z; }
                const bool need_slab = compute && P.z < sv.top_plus_rc;

                Real acc = 0, vs = 0;
                bool core = false;
                uint32_t use = 0;
                Real cterm = 0;
                bool ccore = false;
                if (!ideal) {
                    for (int j0 = 0; j0 < n0; j0 += G) {
                        const int j = j0 + gl;
                        const bool v = compute && j < n0 && j != ex;
                        const Real4 g4 = gas[j < n0 ? j : 0];
                        const Real r2p = dist2(b, P.x, P.y, P.z, g4);
                        const Real r2q = dist2(b, Q.x, Q.y, Q.z, g4);
                        core |= v && r2p < gg.hc2;
                        if (COUNT) use += (uint32_t)(v && r2p < gg.rc2) + (uint32_t)(v && r2q < gg.rc2);
                        acc += v ? lj(r2p, gg) : Real(0);
                        acc -= v ? lj(r2q, gg) : Real(0);
                    }
                    // slab terms at the new position only (the old one's are cached)
                    if (__any(need_slab)) {
                        int cx = 0, cy = 0;
                        if (sv.bins) column_of_lanes(sv, P.x, P.y, cx, cy);
                        for (int k0 = 0; k0 < slab_scan; k0 += G) {
                            const int k = k0 + gl;
                            const bool v = need_slab && k < slab_scan;
                            const int kk = k < slab_scan ? k : 0;
                            const Real4 s4 = sv.atoms[sv.bins ? block_entry(sv, cx, cy, kk) : kk];
                            const Real r2p = dist2(b, P.x, P.y, P.z, s4);
                            core |= v && r2p < gs.hc2;
                            if (COUNT) use += (uint32_t)(v && r2p < gs.rc2);
                            vs += v ? lj(r2p, gs) : Real(0);
                        }
                    }
                    // pair terms with the positions of earlier trials of the batch
                    if (B > 1) {
                        const int g = gl >> 2, k = gl & 3;
                        const int from = (g * G) & (kWave - 1);
                        Real4 X;
                        const Real xp = __shfl(P.x, from), yp = __shfl(P.y, from), zp = __shfl(P.z, from);
                        const Real xq = __shfl(Q.x, from), yq = __shfl(Q.y, from), zq = __shfl(Q.z, from);
                        X.x = k < 2 ? xp : xq; X.y = k < 2 ? yp : yq; X.z = k < 2 ? zp : zq; X.w = 0;
                        const Real4 Y = (k & 1) == 0 ? P : Q;
                        // both positions present (an absent one sits at the far point,
                        // and two absent ones would coincide)
                        const Real zfar = (Real)1.0e3;
                        const bool valid = act && g < grp && X.z < zfar && Y.z < zfar;
                        const Real r2 = dist2(b, Y.x, Y.y, Y.z, X);
                        const Real term = valid ? lj(r2, gg) : Real(0);
                        // the quad's four terms signed and summed: every lane of the quad
                        // holds [phi(P_h-P_g) - phi(Q_h-P_g)] - [phi(P_h-Q_g) - phi(Q_h-Q_g)]
                        cterm = quad_sum((k == 1 || k == 2) ? -term : term);
                        ccore = valid && k == 0 && r2 < gg.hc2;
                    }
                }
                const Real vP = group_sum<G>(vs);                 // slab energy at P
                const Real sde = group_sum<G>(acc) + vP - eo;     // dE on X0
                const uint64_t core_lanes = __ballot(core);
                const uint64_t ccore_lanes = __ballot(ccore);
                const uint32_t packed = (uint32_t)kind | (skip ? 4u : 0u) | (wall ? 8u : 0u) | (compute ? 16u : 0u) |
                                        (need_slab ? 32u : 0u) | ((uint32_t)i << 8);

                // ---- every trial under every outcome of the earlier trials of the batch ----
                // Lane s < 2^h of trial h's group takes the scenario "trial g < h accepted iff
                // bit g of s": N and the changed slots after those trials, h's corrected dE,
                // and h's outcome.  The decisions then follow the one consistent path.
                uint32_t pk[B];
#pragma unroll
                for (int g = 0; g < B; ++g)
                    pk[g] = g < nb ? (uint32_t)__builtin_amdgcn_readlane((int)packed, g * G) : 0u;
                Real cg[B > 1 ? B - 1 : 1];
#pragma unroll
                for (int g = 0; g + 1 < B; ++g) cg[g] = __shfl(cterm, (lane & ~(G - 1)) + 4 * g);
                const uint32_t sc = (uint32_t)gl;
                int ncur = n0;
                uint64_t tmask = 0;          // changed slots, as bits of (slot mod 64)
                double de = (double)sde;
                bool ccr = false;
                // (branch-free: the trial kinds are wave-uniform, the scenarios are not)
#pragma unroll
                for (int g = 0; g + 1 < B; ++g) {
                    const bool take = (g < grp) & (((sc >> g) & 1u) != 0);
                    const int kg = (int)(pk[g] & 3u), ig = (int)(pk[g] >> 8);
                    const uint64_t bi = kg != 1 ? 1ull << (ig & 63) : 0ull;       // moved or refilled slot
                    const uint64_t bn = kg != 0 ? 1ull << ((kg == 1 ? ncur : ncur - 1) & 63) : 0ull;
                    tmask |= take ? (bi | bn) : 0ull;
                    ncur += take ? (kg == 1 ? 1 : (kg == 2 ? -1 : 0)) : 0;
                    de += take ? (double)cg[g] : 0.0;
                    ccr |= take & (((ccore_lanes >> (grp * G + 4 * g)) & 1ull) != 0);
                }
                // (scenarios off the real path may imply an N outside 0..n_max)
                const int nq = ncur < 0 ? 0 : (ncur > n_max ? n_max : ncur);
                const double lq = lnk[kind == 1 ? nq + 1 : nq];
                const bool gcore = ((core_lanes >> (grp * G)) & (G == 64 ? ~0ull : ((1ull << G) - 1))) != 0;
                const bool ichg = ((uint32_t)(((uint64_t)A1 * (uint64_t)(uint32_t)nq) >> 32) != (uint32_t)i) |
                                  (((tmask >> (i & 63)) & 1ull) != 0);
                const bool rk = kind == 1 ? skip & (ncur < n_max) : (n0 == 0 ? ncur > 0 : (ncur > 0) & ichg);
                const bool redo = (sc != 0) & ((compute & gcore) | rk);
                const bool capemp = kind == 1 ? ncur >= n_max : ncur == 0;
                const double th = (kind != 0 && ncur != n0) ? ((kind == 1 ? lnzv_v - lq : lq - lnzv_v) - lnU) * tinv
                                                             : thr;
                const bool cr = compute & (kind != 2) & (gcore | ccr);
                de = compute ? de : 0.0;
                const bool scen = act & (sc < (1u << grp));
                const bool ok = scen & !redo & !capemp & !wall & !cr & (de <= th);
                const uint64_t redo_m = __ballot(scen && redo);
                const uint64_t acc_m = __ballot(ok);
                const uint64_t cap_m = __ballot(scen && !redo && capemp);
                const uint64_t wall_m = __ballot(scen && !redo && !capemp && wall);
                const uint64_t core_m = __ballot(scen && !redo && !capemp && !wall && cr);

                // ---- the path: trial h's scenario is the accept bits of trials 0..h-1 ----
                int nres = 0;
                uint32_t path = 0;
                int nw = n0;                 // N along the path
                for (int h = 0; h < nb; ++h) {
                    const int L0 = h * G + (int)path;
                    if ((redo_m >> L0) & 1ull) break;
                    ++nres;
                    const int kd = (int)(pk[h] & 3u);
                    int ev = -1;
                    if ((cap_m >> L0) & 1ull) ev = kd == 1 ? 6 : 7;
                    else if ((wall_m >> L0) & 1ull) ev = 8;
                    else if ((core_m >> L0) & 1ull) ev = 9;
                    else if ((acc_m >> L0) & 1ull) ev = 2 * kd + 1;
                    stat += (lane == 2 * kd) + (lane == ev);
                    if ((pk[h] & 16u) && ev != 6 && ev != 7 && ev != 8)
                        cand += (uint64_t)(kd == 0 ? 2 : 1) * (uint64_t)(kd == 1 ? nw : nw - 1) +
                                (uint64_t)((pk[h] & 32u) ? slab_scan : 0);
                    if (ev == 2 * kd + 1) {
                        path |= 1u << h;
                        nw += kd == 1 ? 1 : (kd == 2 ? -1 : 0);
                    }
                }
                // the accepted moves of the path, in order
                if (path) {
                    bits |= path << t;
                    for (uint32_t m = path; m; m &= m - 1) {
                        const int h = __builtin_ctz(m);
                        const int L0 = h * G + (int)(path & ((1u << h) - 1u));
                        const int kd = (int)(pk[h] & 3u), is = (int)(pk[h] >> 8);
                        e = in_vgpr(e + bcast(de, L0));
                        // LDS updates in program order (a wave's LDS operations complete in
                        // order); the next pass's reads follow the fence below
                        if (kd == 0) {
                            if (lane == h * G) {
                                gas[is] = P;
                                eslab[is] = vP;
                            }
                        } else if (kd == 1) {
                            if (lane == h * G) {
                                gas[n] = P;
                                eslab[n] = vP;
                            }
                            n += 1;
                        } else {
                            if (lane == 0 && is != n - 1) {
                                gas[is] = gas[n - 1];
                                eslab[is] = eslab[n - 1];
                            }
                            n -= 1;
                        }
                    }
                    wave_sync();
                }
                if (COUNT) useful += grp < nres ? use : 0u;
                t += nres;
            }
            if (tracing && lane == 0)
                a.trace_bits[((size_t)(sweep - a.trace_sweep0) * a.n_walkers + w) * a.trace_words + (t0 >> 5)] = bits;
        }
        // ---- end of sweep: running energy resynchronised, trace N, sample record ----
        if (a.resync_every > 0 && (sweep + 1) % a.resync_every == 0 && !ideal)
            e = full_energy_part<1>(gas, n, sv, b, gg, gs, lane, 0);
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

    {
        double *dst = a.xyz + (size_t)w * a.xyz_stride * 3;
        for (int k = lane; k < n; k += kWave) {
            const Real4 v = gas[k];
            dst[3 * k] = (double)v.x; dst[3 * k + 1] = (double)v.y; dst[3 * k + 2] = (double)v.z;
        }
    }
    {
        uint32_t u = useful;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) u += __shfl_xor(u, o);
        if (lane == 0 && a.pairs) {
            atomicAdd(a.pairs, (unsigned long long)cand);
            atomicAdd(a.pairs + 1, (unsigned long long)u);
        }
    }
    if (lane < kNStat && stat) atomicAdd(a.stats + (size_t)sg * kNStat + lane, (unsigned long long)stat);
    if (lane == 0) {
        a.n[w] = n;
        a.e[w] = e;
    }
}

// ---- batched trials, one wave per trial ---------------------------------------------
// The same decisions as batch_kernel (every trial of a batch evaluated on the
// configuration X0 at the start of the batch, corrected by its pair terms with the
// moves accepted before it, redone in the next pass when an earlier accepted move
// changed what it proposes or assumed), with the B trials of a batch on B waves of one
// workgroup, 64 lanes each.  With one walker per SIMD the single-wave form leaves each
// SIMD one instruction stream; here each SIMD runs one wave of each of four walkers.
// Wave h evaluates trial t + h (its energy on X0, the pair terms with the positions of
// trials 0 .. h-1, and its outcome under each of the 2^h accept patterns of those
// trials, lane s taking pattern s), writes the outcome masks and the scenario energy
// changes into a double-buffered LDS record, and after one barrier every wave walks the
// same path through the records and applies the accepted moves to its own copy of the
// coordinates and slab energies: the copies stay identical, so no second barrier is
// needed before the next pass reads them.
template <bool NEW, bool OLD, bool COUNT>
__device__ __forceinline__ void mw_terms(const Real4 *gas, int n, int ex, const SlabView &sv, const Box &b,
                                         const Pair &gg, const Pair &gs, int lane, bool slab_new, const Real4 &P,
                                         const Real4 &Q, Real &acc, Real &vs, bool &core, uint32_t &use)
{
    // gas: two candidates per lane per step, both loads issued first
    for (int j0 = 0; j0 < n; j0 += 2 * kWave) {
        const int ja = j0 + lane, jb = ja + kWave;
        const Real4 ga = gas[ja < n ? ja : 0];
        const Real4 gb = gas[jb < n ? jb : 0];
        const bool va = ja < n && ja != ex, vb = jb < n && jb != ex;
        if (NEW) {
            const Real ra = dist2(b, P.x, P.y, P.z, ga), rb = dist2(b, P.x, P.y, P.z, gb);
            core |= (va && ra < gg.hc2) || (vb && rb < gg.hc2);
            if (COUNT) use += (uint32_t)(va && ra < gg.rc2) + (uint32_t)(vb && rb < gg.rc2);
            acc += va ? lj(ra, gg) : Real(0);
            acc += vb ? lj(rb, gg) : Real(0);
        }
        if (OLD) {
            const Real ra = dist2(b, Q.x, Q.y, Q.z, ga), rb = dist2(b, Q.x, Q.y, Q.z, gb);
            if (COUNT) use += (uint32_t)(va && ra < gg.rc2) + (uint32_t)(vb && rb < gg.rc2);
            acc -= va ? lj(ra, gg) : Real(0);
            acc -= vb ? lj(rb, gg) : Real(0);
        }
    }
    // slab at the new position only (the old one's is cached)
    if (NEW && slab_new) {
        const int total = sv.bins ? 9 * sv.cap : sv.len;
        int cx = 0, cy = 0;
        if (sv.bins) column_of(sv, P.x, P.y, cx, cy);
        for (int k0 = 0; k0 < total; k0 += 2 * kWave) {
            const int ka = k0 + lane, kb = ka + kWave;
            const bool va = ka < total, vb = kb < total;
            const Real4 sa = sv.atoms[sv.bins ? block_entry(sv, cx, cy, va ? ka : 0) : (va ? ka : 0)];
            const Real4 sb = sv.atoms[sv.bins ? block_entry(sv, cx, cy, vb ? kb : 0) : (vb ? kb : 0)];
            const Real ra = dist2(b, P.x, P.y, P.z, sa), rb = dist2(b, P.x, P.y, P.z, sb);
            core |= (va && ra < gs.hc2) || (vb && rb < gs.hc2);
            if (COUNT) use += (uint32_t)(va && ra < gs.rc2) + (uint32_t)(vb && rb < gs.rc2);
            vs += va ? lj(ra, gs) : Real(0);
            vs += vb ? lj(rb, gs) : Real(0);
        }
    }
}

template <int B, bool COUNT>
__global__ void __launch_bounds__(kWave * B, kSweepWavesPerSimd) mw_kernel(SweepArgs a)
{
    static_assert(B >= 2 && B <= 4, "2 to 4 waves");
    extern __shared__ __align__(32) unsigned char smem[];
    const int h = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);      // this wave's trial in a batch
    const int lane = threadIdx.x % kWave;
    const int blk = blockIdx.x;
    const int cid = a.block_class[blk];
    const ClassDev &C = a.cls[cid];

    const MwLds L = mw_lds(a.max_slab_len, a.gas_stride, B, (int)sizeof(Real));
    Real4 *slab = reinterpret_cast<Real4 *>(smem + L.slab);
    double *lnk = reinterpret_cast<double *>(smem + L.lnk);
    Real4 *gas = reinterpret_cast<Real4 *>(smem + L.gas) + (size_t)h * a.gas_stride;
    Real *eslab = reinterpret_cast<Real *>(smem + L.eslab) + (size_t)h * a.gas_stride;
    double *rec = reinterpret_cast<double *>(smem + L.rec);     // [parity][wave][kMwRecDoubles]

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
    for (int k = threadIdx.x; k < a.gas_stride + 2; k += blockDim.x) lnk[k] = a.lnk[k];
    __syncthreads();

    const int w = a.block_w0[blk];
    const int n_max = C.n_max;
    const int K = C.trials;
    int n = a.n[w];
    double e = a.e[w];
    const int label = a.label[w];
    const int sg = C.state_off + label;
    const double beta = a.beta[sg];
    const double lnz = a.lnz[sg];

    Box b;
    b.lx = in_vgpr((Real)C.lx); b.ly = in_vgpr((Real)C.ly); b.hx = in_vgpr((Real)C.half_lx);
    b.hy = in_vgpr((Real)C.half_ly); b.ix = in_vgpr((Real)C.inv_lx); b.iy = in_vgpr((Real)C.inv_ly);
    Pair gg, gs;
    gg.sig2 = in_vgpr((Real)a.pot.sig2_gg); gg.eps4 = in_vgpr((Real)a.pot.eps4_gg);
    gg.shift = in_vgpr((Real)a.pot.shift_gg); gg.rc2 = in_vgpr((Real)a.pot.rc2); gg.hc2 = in_vgpr((Real)a.pot.hc2_gg);
    gs.sig2 = in_vgpr((Real)a.pot.sig2_gs); gs.eps4 = in_vgpr((Real)a.pot.eps4_gs);
    gs.shift = in_vgpr((Real)a.pot.shift_gs); gs.rc2 = gg.rc2; gs.hc2 = in_vgpr((Real)a.pot.hc2_gs);
    const bool ideal = a.pot.ideal != 0;
    SlabView sv;
    sv.atoms = slab; sv.len = slab_len; sv.bins = C.bins;
    sv.ncx = C.ncx; sv.ncy = C.ncy; sv.cap = C.cap;
    sv.inv_cap = in_vgpr(C.bins ? 1.0f / (float)C.cap : 0.f);
    sv.inv_cw_x = in_vgpr((Real)C.inv_cw_x); sv.inv_cw_y = in_vgpr((Real)C.inv_cw_y);
    sv.top_plus_rc = in_vgpr((Real)(C.slab_top + sqrt(a.pot.rc2)));
    const double lx = in_vgpr(C.lx), ly = in_vgpr(C.ly), zlo = in_vgpr(C.zlo), zhi = in_vgpr(C.zhi);
    const double H = in_vgpr(C.zhi - C.zlo);
    const double md = in_vgpr(a.max_disp);
    const double tinv = in_vgpr(1.0 / beta);
    const double lnzv_v = in_vgpr(lnz + C.lnv);
    const int slab_scan = C.bins ? 9 * C.cap : slab_len;
    Real4 far;                      // a position beyond the cutoff of every atom: absent P or Q
    far.x = 0; far.y = 0; far.z = (Real)1.0e4; far.w = 0;

    // this wave's copy of the coordinates and of each particle's slab energy (computed
    // by every wave with the same arithmetic, so the copies are identical)
    {
        const double *src = a.xyz + (size_t)w * a.xyz_stride * 3;
        for (int k = lane; k < n; k += kWave) {
            Real4 v;
            v.x = (Real)src[3 * k]; v.y = (Real)src[3 * k + 1]; v.z = (Real)src[3 * k + 2]; v.w = 0;
            gas[k] = v;
            Real es = 0;
            if (!ideal && v.z < sv.top_plus_rc) {
                int cx = 0, cy = 0;
                if (sv.bins) column_of_lanes(sv, v.x, v.y, cx, cy);
                for (int q = 0; q < slab_scan; ++q)
                    es += lj(dist2(b, v.x, v.y, v.z, sv.atoms[sv.bins ? block_entry(sv, cx, cy, q) : q]), gs);
            }
            eslab[k] = es;
        }
    }
    wave_sync();

    uint32_t stat = 0;     // wave 0: lane k < kNStat holds counter k
    uint32_t useful = 0;
    uint64_t cand = 0;
    int parity = 0;

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
            const int tn = K - t0 < 32 ? K - t0 : 32;
            uint32_t bits = 0;
            for (int t = 0; t < tn;) {
                const int nb = tn - t < B ? tn - t : B;
                const int n0 = n;
                // ---- every trial of the batch, lane g % B taking trial t + g ----
                const int g = lane % B;
                const bool act = g < nb;
                const int src = 2 * (t + (act ? g : 0));
                const uint32_t A0 = (uint32_t)__shfl((int)R.x, src);
                const uint32_t A1 = (uint32_t)__shfl((int)R.y, src);
                const double ux = __shfl(f0, src), uy = __shfl(f1, src);
                const double uz = __shfl(f2, src + 1), lnU = __shfl(f3, src + 1);
                const int kind = (uint64_t)A0 < a.th_disp ? 0 : ((uint64_t)A0 < a.th_ins ? 1 : 2);
                const bool skip = kind == 1 ? n0 >= n_max : n0 == 0;
                const int i = kind == 1 || skip ? 0 : (int)(((uint64_t)A1 * (uint64_t)n0) >> 32);
                const Real4 o = gas[i];
                const Real eo = kind == 1 || skip ? Real(0) : eslab[i];
                double dx = (double)o.x + md * (2.0 * ux - 1.0);
                double dy = (double)o.y + md * (2.0 * uy - 1.0);
                const double dz = (double)o.z + md * (2.0 * uz - 1.0);
                dx = dx < 0.0 ? dx + lx : (dx >= lx ? dx - lx : dx);
                dy = dy < 0.0 ? dy + ly : (dy >= ly ? dy - ly : dy);
                const double px = kind == 0 ? dx : lx * ux;
                const double py = kind == 0 ? dy : ly * uy;
                const double pz = kind == 0 ? dz : zlo + H * uz;
                const bool wall = (kind == 0) & !skip & ((dz < zlo) | (dz > zhi));
                const double ln0 = lnk[n0], ln1 = lnk[n0 + 1];
                const double c = kind == 0 ? 0.0 : (kind == 1 ? lnzv_v - ln1 : ln0 - lnzv_v);
                const double thr = (c - lnU) * tinv;              // accept iff dE <= thr
                const bool live = act && !skip && !wall;
                const bool compute = live && !ideal;
                Real4 P = far, Q = far;
                if (live && kind != 2) { P.x = (Real)px; P.y = (Real)py; P.z = (Real)pz; }
                if (live && kind != 1) { Q.x = o.x; Q.y = o.y; Q.z = o.z; }
                const uint32_t packed = (uint32_t)kind | (skip ? 4u : 0u) | (wall ? 8u : 0u) |
                                        (compute ? 16u : 0u) | ((compute && kind != 2 && P.z < sv.top_plus_rc) ? 32u : 0u) |
                                        ((uint32_t)i << 8);
                uint32_t pk[B];
#pragma unroll
                for (int q = 0; q < B; ++q) pk[q] = q < nb ? (uint32_t)__builtin_amdgcn_readlane((int)packed, q) : 0u;

                // ---- this wave's trial t + h on X0 ----
                const bool hact = h < nb;
                const uint32_t ph = hact ? (uint32_t)__builtin_amdgcn_readlane((int)packed, h) : 0u;
                const int hkind = (int)(ph & 3u), hi = (int)(ph >> 8);
                const bool hskip = (ph & 4u) != 0, hwall = (ph & 8u) != 0, hcompute = (ph & 16u) != 0;
                const bool hslab = (ph & 32u) != 0;
                Real4 Ph, Qh;
                Ph.x = bcast_real(P.x, h); Ph.y = bcast_real(P.y, h); Ph.z = bcast_real(P.z, h); Ph.w = 0;
                Qh.x = bcast_real(Q.x, h); Qh.y = bcast_real(Q.y, h); Qh.z = bcast_real(Q.z, h); Qh.w = 0;
                const double hthr = bcast(thr, h), hlnU = bcast(lnU, h);
                const uint32_t hA1 = bcast(A1, h);
                const Real heo = bcast_real(eo, h);
                Real acc = 0, vs = 0;
                bool core = false;
                uint32_t use = 0;
                if (hcompute) {
                    const int ex = hkind == 1 ? -1 : hi;
                    if (hkind == 0)
                        mw_terms<true, true, COUNT>(gas, n0, ex, sv, b, gg, gs, lane, hslab, Ph, Qh, acc, vs, core, use);
                    else if (hkind == 1)
                        mw_terms<true, false, COUNT>(gas, n0, ex, sv, b, gg, gs, lane, hslab, Ph, Qh, acc, vs, core, use);
                    else
                        mw_terms<false, true, COUNT>(gas, n0, ex, sv, b, gg, gs, lane, false, Ph, Qh, acc, vs, core, use);
                }
                // pair terms with the positions of the earlier trials: lane 4 q + k holds
                // term k with trial q, the quad's sum
                // [phi(P_h-P_q) - phi(Q_h-P_q)] - [phi(P_h-Q_q) - phi(Q_h-Q_q)] in all four
                Real cterm = 0;
                bool ccore = false;
                if (!ideal && h > 0) {
                    const int q = lane >> 2, k = lane & 3;
                    const int from = q < B ? q : 0;
                    const Real xp = __shfl(P.x, from), yp = __shfl(P.y, from), zp = __shfl(P.z, from);
                    const Real xq = __shfl(Q.x, from), yq = __shfl(Q.y, from), zq = __shfl(Q.z, from);
                    Real4 X;
                    X.x = k < 2 ? xp : xq; X.y = k < 2 ? yp : yq; X.z = k < 2 ? zp : zq; X.w = 0;
                    const Real4 Y = (k & 1) == 0 ? Ph : Qh;
                    const Real zfar = (Real)1.0e3;
                    const bool valid = hact && q < h && X.z < zfar && Y.z < zfar;
                    const Real r2 = dist2(b, Y.x, Y.y, Y.z, X);
                    const Real term = valid ? lj(r2, gg) : Real(0);
                    cterm = quad_sum((k == 1 || k == 2) ? -term : term);
                    ccore = valid && k == 0 && r2 < gg.hc2;
                }
                const Real vP = wave_sum(vs);
                const Real sde = wave_sum(acc) + vP - heo;
                const bool gcore = __ballot(core) != 0ull;
                const uint64_t ccore_lanes = __ballot(ccore);

                // ---- trial h under each accept pattern s (lane s < 2^h) of trials 0 .. h-1 ----
                const uint32_t s = (uint32_t)lane;
                int ncur = n0;
                uint64_t tmask = 0;          // changed slots, as bits of (slot mod 64)
                double de = (double)sde;
                bool ccr = false;
#pragma unroll
                for (int q = 0; q + 1 < B; ++q) {
                    const bool take = (q < h) & (((s >> q) & 1u) != 0);
                    const int kg = (int)(pk[q] & 3u), ig = (int)(pk[q] >> 8);
                    const uint64_t bi = kg != 1 ? 1ull << (ig & 63) : 0ull;
                    const uint64_t bn = kg != 0 ? 1ull << ((kg == 1 ? ncur : ncur - 1) & 63) : 0ull;
                    tmask |= take ? (bi | bn) : 0ull;
                    ncur += take ? (kg == 1 ? 1 : (kg == 2 ? -1 : 0)) : 0;
                    de += take ? (double)bcast_real(cterm, 4 * q) : 0.0;
                    ccr |= take & (((ccore_lanes >> (4 * q)) & 1ull) != 0);
                }
                const int nq = ncur < 0 ? 0 : (ncur > n_max ? n_max : ncur);
                const double lq = lnk[hkind == 1 ? nq + 1 : nq];
                const bool ichg = ((uint32_t)(((uint64_t)hA1 * (uint64_t)(uint32_t)nq) >> 32) != (uint32_t)hi) |
                                  (((tmask >> (hi & 63)) & 1ull) != 0);
                const bool rk = hkind == 1 ? hskip & (ncur < n_max) : (n0 == 0 ? ncur > 0 : (ncur > 0) & ichg);
                const bool redo = (s != 0) & ((hcompute & gcore) | rk);
                const bool capemp = hkind == 1 ? ncur >= n_max : ncur == 0;
                const double th = (hkind != 0 && ncur != n0)
                                      ? ((hkind == 1 ? lnzv_v - lq : lq - lnzv_v) - hlnU) * tinv
                                      : hthr;
                const bool cr = hcompute & (hkind != 2) & (gcore | ccr);
                de = hcompute ? de : 0.0;
                const bool scen = hact & (s < (1u << h));
                const bool ok = scen & !redo & !capemp & !hwall & !cr & (de <= th);
                const uint64_t word = (__ballot(scen && redo) & 0xFFull) | ((__ballot(ok) & 0xFFull) << 8) |
                                      ((__ballot(scen && !redo && capemp) & 0xFFull) << 16) |
                                      ((__ballot(scen && !redo && !capemp && hwall) & 0xFFull) << 24) |
                                      ((__ballot(scen && !redo && !capemp && !hwall && cr) & 0xFFull) << 32);
                double *mine = rec + (size_t)(parity * B + h) * kMwRecDoubles;
                if (lane < 8) mine[lane] = de;
                if (lane == 8) mine[8] = (double)vP;
                if (lane == 9) mine[9] = __longlong_as_double((long long)word);
                __syncthreads();

                // ---- the path, the same in every wave ----
                const double *recs = rec + (size_t)parity * B * kMwRecDoubles;
                int nres = 0;
                uint32_t path = 0;
                int nw = n0;
                for (int q = 0; q < nb; ++q) {
                    // (the same value in every lane: read back as a scalar)
                    const long long wl = __double_as_longlong(recs[q * kMwRecDoubles + 9]);
                    const uint64_t wq = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(wl >> 32)) << 32) |
                                        (uint32_t)__builtin_amdgcn_readfirstlane((int)wl);
                    const int L0 = (int)path;
                    if ((wq >> L0) & 1ull) break;
                    ++nres;
                    const int kd = (int)(pk[q] & 3u);
                    int ev = -1;
                    if ((wq >> (16 + L0)) & 1ull) ev = kd == 1 ? 6 : 7;
                    else if ((wq >> (24 + L0)) & 1ull) ev = 8;
                    else if ((wq >> (32 + L0)) & 1ull) ev = 9;
                    else if ((wq >> (8 + L0)) & 1ull) ev = 2 * kd + 1;
                    if (h == 0) stat += (lane == 2 * kd) + (lane == ev);
                    if ((pk[q] & 16u) && ev != 6 && ev != 7 && ev != 8)
                        cand += (uint64_t)(kd == 0 ? 2 : 1) * (uint64_t)(kd == 1 ? nw : nw - 1) +
                                (uint64_t)((pk[q] & 32u) ? slab_scan : 0);
                    if (ev == 2 * kd + 1) {
                        path |= 1u << q;
                        nw += kd == 1 ? 1 : (kd == 2 ? -1 : 0);
                    }
                }
                if (path) {
                    bits |= path << t;
                    for (uint32_t m = path; m; m &= m - 1) {
                        const int q = __builtin_ctz(m);
                        const int L0 = (int)(path & ((1u << q) - 1u));
                        const int kd = (int)(pk[q] & 3u), is = (int)(pk[q] >> 8);
                        e = in_vgpr(e + recs[q * kMwRecDoubles + L0]);
                        const Real vq = (Real)recs[q * kMwRecDoubles + 8];
                        Real4 Pq;
                        Pq.x = bcast_real(P.x, q); Pq.y = bcast_real(P.y, q); Pq.z = bcast_real(P.z, q); Pq.w = 0;
                        // this wave's copy, in program order (a wave's LDS operations complete in order)
                        if (kd == 0) {
                            if (lane == 0) {
                                gas[is] = Pq;
                                eslab[is] = vq;
                            }
                        } else if (kd == 1) {
                            if (lane == 0) {
                                gas[n] = Pq;
                                eslab[n] = vq;
                            }
                            n += 1;
                        } else {
                            if (lane == 0 && is != n - 1) {
                                gas[is] = gas[n - 1];
                                eslab[is] = eslab[n - 1];
                            }
                            n -= 1;
                        }
                    }
                    wave_sync();
                }
                if (COUNT) useful += h < nres ? use : 0u;
                t += nres;
                parity ^= 1;
            }
            if (tracing && h == 0 && lane == 0)
                a.trace_bits[((size_t)(sweep - a.trace_sweep0) * a.n_walkers + w) * a.trace_words + (t0 >> 5)] = bits;
        }
        // ---- end of sweep: running energy resynchronised (every wave, its own copy), records ----
        if (a.resync_every > 0 && (sweep + 1) % a.resync_every == 0 && !ideal)
            e = full_energy_part<1>(gas, n, sv, b, gg, gs, lane, 0);
        if (h == 0 && lane == 0) {
            if (tracing) a.trace_n[(size_t)(sweep - a.trace_sweep0) * a.n_walkers + w] = n;
            if (a.sample_every > 0 && (sweep + 1) % a.sample_every == 0) {
                const int64_t r = (sweep + 1) / a.sample_every - 1 - a.rec_base;
                const size_t idx = (size_t)r * a.n_walkers + w;
                a.samp_e[idx] = e;
                a.samp_n[idx] = n;
                a.samp_s[idx] = label;
                atomicAdd(a.hist + (size_t)sg * a.hist_stride + n, 1ull);
            }
        }
    }

    if (h == 0) {
        double *dst = a.xyz + (size_t)w * a.xyz_stride * 3;
        for (int k = lane; k < n; k += kWave) {
            const Real4 v = gas[k];
            dst[3 * k] = (double)v.x; dst[3 * k + 1] = (double)v.y; dst[3 * k + 2] = (double)v.z;
        }
    }
    {
        uint32_t u = useful;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) u += __shfl_xor(u, o);
        if (lane == 0 && a.pairs) {
            if (h == 0) atomicAdd(a.pairs, (unsigned long long)cand);
            if (COUNT) atomicAdd(a.pairs + 1, (unsigned long long)u);
        }
    }
    if (h == 0) {
        if (lane < kNStat && stat) atomicAdd(a.stats + (size_t)sg * kNStat + lane, (unsigned long long)stat);
        if (lane == 0) {
            a.n[w] = n;
            a.e[w] = e;
        }
    }
}

// ---- molecular dynamics for the canonical part of the REGC step ----
// Standard normals by Box-Muller: sqrt(-2 ln u1) (cos, sin)(2 pi u2), u open uniforms.
__device__ __forceinline__ void box_muller(uint32_t w1, uint32_t w2, double &z0, double &z1)
{
    const double r = sqrt(-2.0 * log(uniform_open(w1)));
    const double t = 6.283185307179586 * uniform_open(w2);
    z0 = r * cos(t);
    z1 = r * sin(t);
}

__device__ __forceinline__ double md_min_image(double d, double box)
{
    return d > 0.5 * box ? d - box : (d < -0.5 * box ? d + box : d);
}

// Forces on the walker's particles (lane-strided over particles; each particle sums
// its gas partners in index order, then every packed slab entry) and the potential
// energy (FP64, wave-uniform).  Truncated-shifted LJ; the shift does not act on forces.
__device__ double md_forces(const Real4 *gas, int n, const SlabView &sv, const PotDev &pot, const Box &b, double *f,
                            int lane)
{
    double e = 0.0;
    if (!pot.ideal) {
        const double lx = (double)b.lx, ly = (double)b.ly;
        for (int i = lane; i < n; i += kWave) {
            const double xi = (double)gas[i].x, yi = (double)gas[i].y, zi = (double)gas[i].z;
            double fx = 0.0, fy = 0.0, fz = 0.0, ei = 0.0;
            for (int j = 0; j < n; ++j) {
                if (j == i) continue;
                const double dx = md_min_image(xi - (double)gas[j].x, lx);
                const double dy = md_min_image(yi - (double)gas[j].y, ly);
                const double dz = zi - (double)gas[j].z;
                const double r2 = dx * dx + dy * dy + dz * dz;
                if (r2 >= pot.rc2) continue;
                const double s2 = pot.sig2_gg / r2, s6 = s2 * s2 * s2;
                const double g = 6.0 * pot.eps4_gg * (2.0 * s6 * s6 - s6) / r2;
                fx += g * dx; fy += g * dy; fz += g * dz;
                ei += 0.5 * (pot.eps4_gg * (s6 * s6 - s6) - pot.shift_gg);
            }
            const int ns = sv.bins ? sv.ncx * sv.ncy * sv.cap : sv.len;
            for (int k = 0; k < ns; ++k) {
                const Real4 sa = sv.atoms[k];
                const double dx = md_min_image(xi - (double)sa.x, lx);
                const double dy = md_min_image(yi - (double)sa.y, ly);
                const double dz = zi - (double)sa.z;
                const double r2 = dx * dx + dy * dy + dz * dz;
                if (r2 >= pot.rc2) continue;
                const double s2 = pot.sig2_gs / r2, s6 = s2 * s2 * s2;
                const double g = 6.0 * pot.eps4_gs * (2.0 * s6 * s6 - s6) / r2;
                fx += g * dx; fy += g * dy; fz += g * dz;
                ei += pot.eps4_gs * (s6 * s6 - s6) - pot.shift_gs;
            }
            f[3 * i] = fx; f[3 * i + 1] = fy; f[3 * i + 2] = fz;
            e += ei;
        }
    } else {
        for (int i = lane; i < n; i += kWave) f[3 * i] = f[3 * i + 1] = f[3 * i + 2] = 0.0;
    }
    wave_sync();
    return wave_sum(e);
}

// md_steps velocity-Verlet steps with the stochastic velocity-rescaling thermostat
// (Bussi, Donadio, Parrinello 2007): K' = c K + (1-c) Kbar (R1^2 + S)/Nf
// + 2 sqrt(c (1-c) K Kbar / Nf) R1 with c = exp(-dt/tau), Kbar = Nf T / 2, Nf = 3N,
// R1 from Philox block (1 + step, q, walker, 2) words (0,1), S the squares of the
// first Nf - 1 normals of blocks (1 + step, q, walker, 16 + b) (four per block).
// Returns the potential energy of the final configuration.
__device__ double md_run(Real4 *gas, double *v, double *f, int n, double T, const SlabView &sv, const PotDev &pot,
                         const Box &b, double zlo, double zhi, const PaperArgs &pa, int64_t q, int w, uint32_t k0,
                         uint32_t k1, int lane)
{
    const double dt = pa.md_dt, lx = (double)b.lx, ly = (double)b.ly;
    double e = md_forces(gas, n, sv, pot, b, f, lane);
    for (int st = 0; st < pa.md_steps; ++st) {
        for (int i = lane; i < n; i += kWave) {
            double *u = v + 3 * i;
            const double *g = f + 3 * i;
            u[0] += 0.5 * dt * g[0]; u[1] += 0.5 * dt * g[1]; u[2] += 0.5 * dt * g[2];
            double px = (double)gas[i].x + dt * u[0], py = (double)gas[i].y + dt * u[1], pz = (double)gas[i].z + dt * u[2];
            if (px < 0.0) px += lx; else if (px >= lx) px -= lx;
            if (py < 0.0) py += ly; else if (py >= ly) py -= ly;
            if (pz < zlo) { pz = 2.0 * zlo - pz; u[2] = -u[2]; }
            else if (pz > zhi) { pz = 2.0 * zhi - pz; u[2] = -u[2]; }
            Real4 nv; nv.x = (Real)px; nv.y = (Real)py; nv.z = (Real)pz; nv.w = 0;
            gas[i] = nv;
        }
        wave_sync();
        e = md_forces(gas, n, sv, pot, b, f, lane);
        double kin = 0.0;
        for (int i = lane; i < n; i += kWave) {
            double *u = v + 3 * i;
            const double *g = f + 3 * i;
            u[0] += 0.5 * dt * g[0]; u[1] += 0.5 * dt * g[1]; u[2] += 0.5 * dt * g[2];
            kin += 0.5 * u[0] * u[0] + 0.5 * u[1] * u[1] + 0.5 * u[2] * u[2];
        }
        if (pa.md_tau > 0.0) {
            const double K = wave_sum(kin);
            if (K > 0.0) {
                const int nf = 3 * n;
                const uint4 R = philox4x32_10(make_uint4((uint32_t)(1 + st), (uint32_t)q, (uint32_t)w, 2u), k0, k1);
                double r1, unused;
                box_muller(R.x, R.y, r1, unused);
                double s = 0.0;
                for (int blk = lane; 4 * blk < nf - 1; blk += kWave) {
                    const uint4 Q = philox4x32_10(make_uint4((uint32_t)(1 + st), (uint32_t)q, (uint32_t)w,
                                                             16u + (uint32_t)blk), k0, k1);
                    double z[4];
                    box_muller(Q.x, Q.y, z[0], z[1]);
                    box_muller(Q.z, Q.w, z[2], z[3]);
                    for (int k = 0; k < 4 && 4 * blk + k < nf - 1; ++k) s += z[k] * z[k];
                }
                const double S = wave_sum(s);
                const double Kbar = 0.5 * nf * T;
                const double c = exp(-dt / pa.md_tau);
                const double K2 = c * K + (1.0 - c) * Kbar * (r1 * r1 + S) / nf +
                                  2.0 * sqrt(c * (1.0 - c) * K * Kbar / nf) * r1;
                const double alpha = sqrt(K2 / K);
                for (int k = lane; k < nf; k += kWave) v[k] *= alpha;
            }
        }
        wave_sync();
    }
    return e;
}

// The paper's REGC step (Sec. II.A; Sec. III.A for the LJ run): for each step the
// coin of Philox block (0, step, 0xFFFFFFFF - class, 6) -- open uniform of word 0
// below x0 -- selects one particle-exchange attempt per walker (trial 0: removal
// when A0 < 2^31, i.e. y1 < 1/2, else insertion); otherwise the host has run the
// replica-exchange step before this launch.  Then mc_cycles cycles of N
// displacement attempts, trials 1 .. mc_cycles N with N after trial 0.  Same
// trial arithmetic as sweep_kernel (one wave per walker).  Single-class contexts.
__global__ void __launch_bounds__(kWave * kMaxWalkersPerBlock) paper_kernel(SweepArgs a, PaperArgs pa)
{
    extern __shared__ __align__(32) unsigned char smem[];
    const int wave = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    const int waves = blockDim.x / kWave;
    const int blk = blockIdx.x;
    const ClassDev &C = a.cls[0];
    const int nw = a.block_nw[blk];

    const LdsLayout L = lds_layout(a.max_slab_len, a.gas_stride, a.max_slab_scan, waves, 0,
                                   (int)sizeof(Real));
    Real4 *slab = reinterpret_cast<Real4 *>(smem + L.slab);
    double *lnk = reinterpret_cast<double *>(smem + L.lnk);
    Real4 *gas = reinterpret_cast<Real4 *>(smem + L.gas) + (size_t)wave * a.gas_stride;
    const bool use_md = pa.md_steps > 0;
    double *mdv = reinterpret_cast<double *>(smem + lds_round(L.total)) + (size_t)wave * a.gas_stride * 6;
    double *mdf = mdv + (size_t)a.gas_stride * 3;

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
    for (int k = threadIdx.x; k < a.gas_stride + 2; k += blockDim.x) lnk[k] = a.lnk[k];
    __syncthreads();
    if (wave >= nw) return;

    const int w = a.block_w0[blk] + wave;
    double tv = use_md ? pa.tv[w] : 0.0;
    const int n_max = C.n_max;
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
        if (use_md)
            for (int k = lane; k < 3 * n; k += kWave) mdv[k] = pa.vel[(size_t)w * a.xyz_stride * 3 + k];
    }
    wave_sync();

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
    const int slab_scan = C.bins ? 9 * C.cap : slab_len;

    uint32_t stat = 0;
    uint32_t useful = 0;
    uint64_t cand = 0;
    for (int it = 0; it < a.n_sweeps; ++it) {
        const int64_t step = a.sweep0 + it;
        const bool tracing = a.trace_bits != nullptr && (step - a.trace_sweep0) < a.trace_cap &&
                             step >= a.trace_sweep0;
        const uint4 coin = philox4x32_10(make_uint4(0u, (uint32_t)step, 0xFFFFFFFFu, 6u), a.key0, a.key1);
        const bool exchange = uniform_open(coin.x) < pa.x0;
        if (use_md) {
            // velocities: drawn at the state's T when none exist, rescaled after a change of T
            const double Tw = 1.0 / beta;
            if (tv == 0.0) {
                for (int i = lane; i < n; i += kWave) {
                    const uint4 R = philox4x32_10(make_uint4(0x80000000u + (uint32_t)i, (uint32_t)step, (uint32_t)w, 4u),
                                                  a.key0, a.key1);
                    double z0, z1, z2, z3;
                    box_muller(R.x, R.y, z0, z1);
                    box_muller(R.z, R.w, z2, z3);
                    mdv[3 * i] = sqrt(Tw) * z0; mdv[3 * i + 1] = sqrt(Tw) * z1; mdv[3 * i + 2] = sqrt(Tw) * z2;
                }
            } else if (tv != Tw) {
                const double sc = sqrt(Tw / tv);
                for (int k = lane; k < 3 * n; k += kWave) mdv[k] *= sc;
            }
            tv = Tw;
            wave_sync();
        }
        const int n_before = n;
        int i_removed = -1;
        int T = use_md ? 1 : 1 + pa.mc_cycles * n;
        for (int t0 = 0; t0 < T; t0 += 32) {
            const uint4 R = philox4x32_10(
                make_uint4((uint32_t)(t0 + (lane >> 1)), (uint32_t)step, (uint32_t)w, (uint32_t)(lane & 1)),
                a.key0, a.key1);
            const double f0 = uniform_open(R.z), f1 = uniform_open(R.w), f2 = uniform_open(R.x);
            const double f3 = log(uniform53(R.y, R.z));
            uint32_t bits = 0;
            for (int tt = 0; tt < 32 && t0 + tt < T; ++tt) {
                const int t = t0 + tt;
                if (t == 0 && !exchange) continue;
                const uint32_t A0 = bcast(R.x, 2 * tt), A1 = bcast(R.y, 2 * tt);
                // trial 0: removal when y1 = A0 / 2^32 < 1/2, else insertion; then displacements
                const int kind = t == 0 ? (A0 < 0x80000000u ? 2 : 1) : 0;
                stat += lane == 2 * kind;
                bool accepted = false;
                if (kind == 1 ? n >= n_max : n == 0) {
                    stat += lane == (kind == 1 ? 6 : 7);
                } else {
                    const double lnU = bcast(f3, 2 * tt + 1);
                    const double ux = bcast(f0, 2 * tt), uy = bcast(f1, 2 * tt), uz = bcast(f2, 2 * tt + 1);
                    const int i = kind == 1 ? -1 : (int)(((uint64_t)A1 * (uint64_t)n) >> 32);
                    const Real4 o = gas[kind == 1 ? 0 : i];
                    double px = 0.0, py = 0.0, pz = 0.0, c;
                    bool wall = false;
                    if (kind == 0) {
                        px = (double)o.x + md * (2.0 * ux - 1.0);
                        py = (double)o.y + md * (2.0 * uy - 1.0);
                        pz = (double)o.z + md * (2.0 * uz - 1.0);
                        if (px < 0.0) px += lx; else if (px >= lx) px -= lx;
                        if (py < 0.0) py += ly; else if (py >= ly) py -= ly;
                        wall = pz < zlo || pz > zhi;
                        c = 0.0;
                    } else if (kind == 1) {
                        px = lx * ux;
                        py = ly * uy;
                        pz = zlo + H * uz;
                        c = lnzv - lnk[n + 1];
                    } else {
                        c = lnk[n] - lnzv;
                    }
                    if (wall) {
                        stat += lane == 8;
                    } else {
                        const double thr = (c - lnU) * tinv;
                        const Real qx = (Real)px, qy = (Real)py, qz = (Real)pz;
                        double de = 0.0;
                        bool core = false;
                        if (!ideal) {
                            Real pd;
                            if (kind == 0)
                                pd = partial_delta<true, true, 1, false>(gas, n, i, sv, b, gg, gs, lane, 0, qx, qy, qz,
                                                                         o.x, o.y, o.z, nullptr, nullptr, core,
                                                                         useful);
                            else if (kind == 1)
                                pd = partial_delta<true, false, 1, false>(gas, n, -1, sv, b, gg, gs, lane, 0, qx, qy,
                                                                          qz, qx, qy, qz, nullptr, nullptr, core,
                                                                          useful);
                            else
                                pd = partial_delta<false, true, 1, false>(gas, n, i, sv, b, gg, gs, lane, 0, o.x, o.y,
                                                                          o.z, o.x, o.y, o.z, nullptr, nullptr, core,
                                                                          useful);
                            de = (double)pd;
                            const uint64_t mult = kind == 0 ? 2 : 1;
                            const Real zmin = kind == 0 ? (qz < o.z ? qz : o.z) : (kind == 1 ? qz : o.z);
                            cand += mult * (uint64_t)((kind == 1 ? n : n - 1) +
                                                      (zmin < sv.top_plus_rc ? slab_scan : 0));
                        }
                        if (core && kind != 2) {
                            stat += lane == 9;
                        } else if (de <= thr) {
                            accepted = true;
                            stat += lane == 2 * kind + 1;
                            e += de;
                            if (kind == 0) {
                                if (lane == 0) {
                                    Real4 v; v.x = qx; v.y = qy; v.z = qz; v.w = 0;
                                    gas[i] = v;
                                }
                            } else if (kind == 1) {
                                if (lane == 0) {
                                    Real4 v; v.x = qx; v.y = qy; v.z = qz; v.w = 0;
                                    gas[n] = v;
                                }
                                n += 1;
                            } else {
                                if (lane == 0 && i != n - 1) gas[i] = gas[n - 1];
                                i_removed = i;
                                n -= 1;
                            }
                        }
                    }
                }
                if (accepted) {
                    bits |= 1u << tt;
                    wave_sync();
                }
                if (t == 0 && !use_md) T = 1 + pa.mc_cycles * n;      // N after the exchange attempt
            }
            if (tracing && lane == 0)
                a.trace_bits[((size_t)(step - a.trace_sweep0) * a.n_walkers + w) * a.trace_words + (t0 >> 5)] = bits;
        }
        if (use_md) {
            // the inserted particle's velocity (Philox block (0, step, walker, 3)); the
            // removed slot takes the last particle's; then the MD run
            const double Tw = 1.0 / beta;
            if (n > n_before && lane == 0) {
                const uint4 R = philox4x32_10(make_uint4(0u, (uint32_t)step, (uint32_t)w, 3u), a.key0, a.key1);
                double z0, z1, z2, z3;
                box_muller(R.x, R.y, z0, z1);
                box_muller(R.z, R.w, z2, z3);
                mdv[3 * n_before] = sqrt(Tw) * z0; mdv[3 * n_before + 1] = sqrt(Tw) * z1;
                mdv[3 * n_before + 2] = sqrt(Tw) * z2;
            } else if (n < n_before && lane == 0 && i_removed != n_before - 1) {
                for (int k = 0; k < 3; ++k) mdv[3 * i_removed + k] = mdv[3 * (n_before - 1) + k];
            }
            wave_sync();
            if (n > 0) e = md_run(gas, mdv, mdf, n, Tw, sv, a.pot, b, zlo, zhi, pa, step, w, a.key0, a.key1, lane);
        }
        if (lane == 0) {
            if (tracing) {
                // the words past this step's last trial hold no trial
                uint32_t *row = a.trace_bits + ((size_t)(step - a.trace_sweep0) * a.n_walkers + w) * a.trace_words;
                for (int wd = (T + 31) / 32; wd < a.trace_words; ++wd) row[wd] = 0u;
                a.trace_n[(size_t)(step - a.trace_sweep0) * a.n_walkers + w] = n;
            }
            if (a.sample_every > 0 && (step + 1) % a.sample_every == 0) {
                const int64_t rec = (step + 1) / a.sample_every - 1 - a.rec_base;
                const size_t idx = (size_t)rec * a.n_walkers + w;
                a.samp_e[idx] = e;
                a.samp_n[idx] = n;
                a.samp_s[idx] = label;
                atomicAdd(a.hist + (size_t)sg * a.hist_stride + n, 1ull);
            }
        }
    }

    {
        double *dst = a.xyz + (size_t)w * a.xyz_stride * 3;
        for (int k = lane; k < n; k += kWave) {
            const Real4 v = gas[k];
            dst[3 * k] = (double)v.x; dst[3 * k + 1] = (double)v.y; dst[3 * k + 2] = (double)v.z;
        }
        if (use_md) {
            for (int k = lane; k < 3 * n; k += kWave) pa.vel[(size_t)w * a.xyz_stride * 3 + k] = mdv[k];
            if (lane == 0) pa.tv[w] = tv;
        }
    }
    if (lane == 0 && a.pairs) atomicAdd(a.pairs, (unsigned long long)cand);
    if (lane < kNStat && stat) atomicAdd(a.stats + (size_t)sg * kNStat + lane, (unsigned long long)stat);
    if (lane == 0) {
        a.n[w] = n;
        a.e[w] = e;
    }
}

// Full recomputation of each walker's energy (gas-gas pairs once, gas-slab for
// every atom), pair terms in Real, sums in FP64.  One wavefront per walker.
__global__ void __launch_bounds__(256) ENERGY_KERNEL(EnergyArgs a)
{
    const int w = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    if (w >= a.n_walkers) return;
    const int cid = a.walker_class[w];
    const ClassDev &C = a.cls[cid];
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

}  // namespace fp64 / fp32

#if defined(REGC_FP64)
using namespace fp64;
#else
using namespace fp32;
#endif

hipError_t ENERGY_LAUNCH(const EnergyArgs &a, hipStream_t s)
{
    const int per = 4;
    hipLaunchKernelGGL(ENERGY_KERNEL, dim3((a.n_walkers + per - 1) / per), dim3(kWave * per), 0, s, a);
    return hipGetLastError();
}

hipError_t PAPER_LAUNCH(const SweepArgs &a, const PaperArgs &p, int n_blocks, int waves_per_block, size_t smem,
                        hipStream_t s)
{
    hipLaunchKernelGGL(paper_kernel, dim3(n_blocks), dim3(kWave * waves_per_block), smem, s, a, p);
    return hipGetLastError();
}

hipError_t SWEEP_LAUNCH(const SweepArgs &a, int n_blocks, int waves_per_block, int split, bool cull, int batch,
                        size_t smem, hipStream_t s)
{
    const dim3 grid(n_blocks), block(kWave * waves_per_block);
    if (batch == 4 && split == 4) {
        if (a.count_pairs) hipLaunchKernelGGL((mw_kernel<4, true>), grid, block, smem, s, a);
        else hipLaunchKernelGGL((mw_kernel<4, false>), grid, block, smem, s, a);
    } else if (batch == 2 && split == 2) {
        if (a.count_pairs) hipLaunchKernelGGL((mw_kernel<2, true>), grid, block, smem, s, a);
        else hipLaunchKernelGGL((mw_kernel<2, false>), grid, block, smem, s, a);
    } else if (batch == 4) {
        if (a.count_pairs) hipLaunchKernelGGL((batch_kernel<4, true>), grid, block, smem, s, a);
        else hipLaunchKernelGGL((batch_kernel<4, false>), grid, block, smem, s, a);
    } else if (batch == 2) {
        if (a.count_pairs) hipLaunchKernelGGL((batch_kernel<2, true>), grid, block, smem, s, a);
        else hipLaunchKernelGGL((batch_kernel<2, false>), grid, block, smem, s, a);
    } else if (split == 4) {
        if (cull) hipLaunchKernelGGL((sweep_kernel<4, true>), grid, block, smem, s, a);
        else hipLaunchKernelGGL((sweep_kernel<4, false>), grid, block, smem, s, a);
    } else if (split == 2) {
        if (cull) hipLaunchKernelGGL((sweep_kernel<2, true>), grid, block, smem, s, a);
        else hipLaunchKernelGGL((sweep_kernel<2, false>), grid, block, smem, s, a);
    } else {
        if (cull) hipLaunchKernelGGL((sweep_kernel<1, true>), grid, block, smem, s, a);
        else hipLaunchKernelGGL((sweep_kernel<1, false>), grid, block, smem, s, a);
    }
    return hipGetLastError();
}

static const void *persist_kernel(int split)
{
    return split == 2 ? reinterpret_cast<const void *>(&sweep_persist_kernel<2>)
                      : reinterpret_cast<const void *>(&sweep_persist_kernel<1>);
}

hipError_t PERSIST_LAUNCH(const SweepArgs &a, int n_blocks, int waves_per_block, int split, size_t smem,
                          hipStream_t s)
{
    SweepArgs arg = a;
    void *args[] = {&arg};
    return hipLaunchCooperativeKernel(persist_kernel(split), dim3(n_blocks), dim3(kWave * waves_per_block), args,
                                      (unsigned)smem, s);
}

hipError_t PERSIST_CAPACITY(int waves_per_block, int split, size_t smem, int *max_blocks)
{
    int dev = 0, n_cu = 0, per = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, persist_kernel(split), kWave * waves_per_block, smem);
    *max_blocks = per * n_cu;
    return e;
}

}  // namespace regc
