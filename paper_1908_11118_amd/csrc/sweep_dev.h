// sweep_dev.h -- device helpers of the REGC trial kernels (pair terms, wave
// reductions, slab access, the energy change of a trial), included by the
// sampling kernels.  Each including file is compiled once per precision
// (-DREGC_FP64 or -DREGC_FP32); the helpers then live in namespace
// regc::fp64 or regc::fp32 with Real = double or float.
#pragma once
#include "regc_dev.h"
#include "philox_dev.h"

namespace regc {

// Each compilation gets its own namespace: the kernels are templates
// with the same names in both precisions, and one symbol per precision must reach
// the code-object registry.
#if defined(REGC_FP64)
#define REGC_PREC fp64
#elif defined(REGC_FP32)
#define REGC_PREC fp32
#else
#error "compile with -DREGC_FP64 or -DREGC_FP32"
#endif

namespace REGC_PREC {
#if defined(REGC_FP64)
typedef double Real;
struct alignas(32) Real4 { double x, y, z, w; };
#else
typedef float Real;
struct alignas(16) Real4 { float x, y, z, w; };
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

// truncated-shifted LJ 12-6 at squared distance r2 (r2 < rc2 is the caller's business)
__device__ __forceinline__ Real lj_inside(Real r2, Real sig2, Real eps4, Real shift)
{
#if defined(REGC_FP64)
    const double s2 = sig2 / r2;
#else
    const float s2 = sig2 * __builtin_amdgcn_rcpf(r2);
#endif
    const Real s6 = s2 * s2 * s2;
    return eps4 * (s6 * s6 - s6) - shift;
}

__device__ __forceinline__ Real lj(Real r2, const Pair &p)
{
    const Real v = lj_inside(r2, p.sig2, p.eps4, p.shift);
    return r2 < p.rc2 ? v : Real(0);
}

// Wave-wide sum with DPP (quad permutes, row mirrors, row broadcasts); the total
// ends in lane 63 and is read back as a wave-uniform value.  The order of the
// additions is fixed, so the result is deterministic.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f32(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ float wave_sum(float v)
{
    v += dpp_f32<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
    v += dpp_f32<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
    v += dpp_f32<0x141, 0xF>(v);   // row_half_mirror
    v += dpp_f32<0x140, 0xF>(v);   // row_mirror
    v += dpp_f32<0x142, 0xA>(v);   // row_bcast:15 into rows 1, 3
    v += dpp_f32<0x143, 0xC>(v);   // row_bcast:31 into rows 2, 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_f64<0xB1, 0xF>(v);
    v += dpp_f64<0x4E, 0xF>(v);
    v += dpp_f64<0x141, 0xF>(v);
    v += dpp_f64<0x140, 0xF>(v);
    v += dpp_f64<0x142, 0xA>(v);
    v += dpp_f64<0x143, 0xC>(v);
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

// Sum over each quad of lanes (4 lanes), the total in every lane of the quad.
__device__ __forceinline__ float quad_sum(float v)
{
    v += dpp_f32<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
    v += dpp_f32<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
    return v;
}

__device__ __forceinline__ double quad_sum(double v)
{
    v += dpp_f64<0xB1, 0xF>(v);
    v += dpp_f64<0x4E, 0xF>(v);
    return v;
}

// Sum over aligned groups of G lanes (16, 32 or 64), the total in every lane of the
// group; the order of the additions is fixed (DPP within rows of 16, then across rows).
template <int G>
__device__ __forceinline__ float group_sum(float v)
{
    v += dpp_f32<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
    v += dpp_f32<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
    v += dpp_f32<0x141, 0xF>(v);   // row_half_mirror
    v += dpp_f32<0x140, 0xF>(v);   // row_mirror: every lane holds its row's sum
    if (G >= 32) v += __shfl_xor(v, 16);
    if (G >= 64) v += __shfl_xor(v, 32);
    return v;
}

template <int G>
__device__ __forceinline__ double group_sum(double v)
{
    v += dpp_f64<0xB1, 0xF>(v);
    v += dpp_f64<0x4E, 0xF>(v);
    v += dpp_f64<0x141, 0xF>(v);
    v += dpp_f64<0x140, 0xF>(v);
    if (G >= 32) v += __shfl_xor(v, 16);
    if (G >= 64) v += __shfl_xor(v, 32);
    return v;
}

// A condition that every lane of the wave holds alike, as a wave-uniform value: the
// branch on it is a scalar branch.
__device__ __forceinline__ bool uniform(bool c)
{
    return __builtin_amdgcn_readfirstlane((int)c) != 0;
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Keep a wave-uniform constant in a VGPR: the hot loop has more uniform values
// than SGPRs, and VALU operands read from VGPRs cost no scalar-register spills.
template <typename T>
__device__ __forceinline__ T in_vgpr(T x)
{
    asm volatile("" : "+v"(x));
    return x;
}

__device__ __forceinline__ uint32_t bcast(uint32_t v, int lane)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

__device__ __forceinline__ double bcast(double v, int lane)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ float bcast(float v, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

__device__ __forceinline__ Real bcast_real(Real v, int lane) { return bcast(v, lane); }

// Slab access: all atoms, or the 3x3 block of x-y columns around a column
// (periodic in x and y; column ids row-major, y outer).
struct SlabView {
    const Real4 *atoms;
    int len;                  // entries when unbinned
    int bins, ncx, ncy, cap;
    float inv_cap;
    Real inv_cw_x, inv_cw_y;
    Real top_plus_rc;
};

// Column (cx, cy) of a position, clamped to the grid; the caller's position is
// wave-uniform, so the result is moved to scalar registers.
__device__ __forceinline__ void column_of(const SlabView &sv, Real x, Real y, int &cx, int &cy)
{
    const int ix = (int)(x * sv.inv_cw_x);
    const int iy = (int)(y * sv.inv_cw_y);
    cx = __builtin_amdgcn_readfirstlane(ix < 0 ? 0 : (ix >= sv.ncx ? sv.ncx - 1 : ix));
    cy = __builtin_amdgcn_readfirstlane(iy < 0 ? 0 : (iy >= sv.ncy ? sv.ncy - 1 : iy));
}

// Column of a position as a per-lane value (positions that differ between lanes).
__device__ __forceinline__ void column_of_lanes(const SlabView &sv, Real x, Real y, int &cx, int &cy)
{
    const int ix = (int)(x * sv.inv_cw_x);
    const int iy = (int)(y * sv.inv_cw_y);
    cx = ix < 0 ? 0 : (ix >= sv.ncx ? sv.ncx - 1 : ix);
    cy = iy < 0 ? 0 : (iy >= sv.ncy ? sv.ncy - 1 : iy);
}

// Periodic neighbour c + d (d in -1..1) of a column index in [0, nc): as an
// unsigned value, -1 wraps to the largest integer and min() picks nc - 1, and
// nc becomes 0 the same way.
__device__ __forceinline__ uint32_t wrap_col(int c, int d, int nc)
{
    uint32_t u = (uint32_t)(c + d);
    u = min(u, u + (uint32_t)nc);
    return min(u, u - (uint32_t)nc);
}

// Slab entry kk (0 <= kk < 9 cap) of the 3x3 column block around column (cx, cy):
// slot kk % cap of the block's column sp = kk / cap, sp = 3 (dy + 1) + (dx + 1).
__device__ __forceinline__ int block_entry(const SlabView &sv, int cx, int cy, int kk)
{
    const int sp = (int)(((float)kk + 0.5f) * sv.inv_cap);
    const int q = (sp * 11) >> 5;   // sp / 3 for sp in 0..8
    const uint32_t ux = wrap_col(cx, sp - 3 * q - 1, sv.ncx);
    const uint32_t uy = wrap_col(cy, q - 1, sv.ncy);
    return (int)((uy * (uint32_t)sv.ncx + ux) * (uint32_t)sv.cap) + (kk - sp * sv.cap);
}

// This wave's part (wave `part` of SPLIT) of the walker's total energy: every gas
// pair once and every gas atom against the slab entries that can lie within the
// cutoff (its column block, or all entries when unbinned), pair terms in Real,
// per-lane sums in FP64.  Returns the wave-uniform partial sum.
template <int SPLIT>
__device__ double full_energy_part(const Real4 *gas, int n, const SlabView &sv, const Box &b, const Pair &gg,
                                   const Pair &gs, int lane, int part)
{
    double acc = 0.0;
    const int total = sv.bins ? 9 * sv.cap : sv.len;
    for (int i = 0; i < n; ++i) {
        const Real4 p = gas[i];
        for (int j = i + 1 + part * kWave + lane; j < n; j += SPLIT * kWave)
            acc += (double)lj(dist2(b, p.x, p.y, p.z, gas[j]), gg);
        if (p.z < sv.top_plus_rc) {
            int cx = 0, cy = 0;
            if (sv.bins) column_of(sv, p.x, p.y, cx, cy);
            for (int k = part * kWave + lane; k < total; k += SPLIT * kWave) {
                const int idx = sv.bins ? block_entry(sv, cx, cy, k) : k;
                acc += (double)lj(dist2(b, p.x, p.y, p.z, sv.atoms[idx]), gs);
            }
        }
    }
    return wave_sum(acc);
}

// Appends the lanes' values whose predicate holds to an LDS queue (wave-wide
// compaction): each lane's slot is the number of set predicate bits below it.
__device__ __forceinline__ void push(Real *queue, int &count, bool pred, Real value)
{
    const uint64_t mask = __ballot(pred);
    const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
    if (pred) queue[count + (int)below] = value;
    count += __popcll(mask);
}

// One candidate atom g (mask m): pair terms of the new position p (NEW, added) and
// of the old position q (OLD, subtracted).  CULL queues the in-cutoff squared
// distances (old ones negated) instead of evaluating them.
template <bool NEW, bool OLD, bool CULL>
__device__ __forceinline__ void candidate(const Box &b, const Pair &pp, bool m, const Real4 &g, Real px, Real py,
                                          Real pz, Real qx, Real qy, Real qz, Real &acc, bool &core,
                                          uint32_t &useful, Real *queue, int &count)
{
    if (NEW) {
        const Real r2 = dist2(b, px, py, pz, g);
        core |= m && r2 < pp.hc2;
        if (CULL) {
            push(queue, count, m && r2 < pp.rc2, r2);
        } else {
            useful += m && r2 < pp.rc2;
            acc += m ? lj(r2, pp) : Real(0);
        }
    }
    if (OLD) {
        const Real r2 = dist2(b, qx, qy, qz, g);
        if (CULL) {
            push(queue, count, m && r2 < pp.rc2, -r2);
        } else {
            useful += m && r2 < pp.rc2;
            acc -= m ? lj(r2, pp) : Real(0);
        }
    }
}

// This wave's part of the energy change of a trial: sum over the other gas atoms
// (all j < n except `skip`) and over the slab candidates of phi(|p - r|) (NEW)
// minus phi(|q - r|) (OLD).  The wave with index `part` of SPLIT takes every
// SPLIT-th block of candidates; trip counts are wave-uniform.  Returns the
// wave-uniform partial sum; `core_out` is this wave's hard-core flag.  PRE (one wave
// per walker): `pre` holds the first step's two gas atoms per lane, read by the caller.
template <bool NEW, bool OLD, int SPLIT, bool CULL, bool PRE = false>
__device__ __forceinline__ Real partial_delta(const Real4 *gas, int n, int skip, const SlabView &sv, const Box &b,
                                              const Pair &gg, const Pair &gs, int lane, int part, Real px, Real py,
                                              Real pz, Real qx, Real qy, Real qz, Real *qgas, Real *qslab,
                                              bool &core_out, uint32_t &useful, const Real4 *pre = nullptr)
{
    constexpr int U = SPLIT == 1 ? 2 : 1;   // candidates per lane per step
    constexpr int STEP = SPLIT * U * kWave;
    Real acc = 0;
    bool core = false;
    int ng = 0, ns = 0;
    if (SPLIT == 2 && uniform(n > STEP && n <= 2 * STEP)) {
        // two blocks for this wave (more than 128 atoms, two waves): both reads issued
        // before the terms, one LDS round trip instead of two on the trial's chain (the
        // walkers with the most atoms are the last to finish a launch)
        const int j = part * kWave + lane, j2 = j + STEP;
        const bool v1 = j < n, v2 = j2 < n;
        const Real4 ga = gas[v1 ? j : 0];
        const Real4 gb = gas[v2 ? j2 : 0];
        candidate<NEW, OLD, CULL>(b, gg, v1 && j != skip, ga, px, py, pz, qx, qy, qz, acc, core, useful, qgas, ng);
        candidate<NEW, OLD, CULL>(b, gg, v2 && j2 != skip, gb, px, py, pz, qx, qy, qz, acc, core, useful, qgas, ng);
    } else
    for (int j0 = part * U * kWave; j0 < n; j0 += STEP) {
        if (PRE && j0 == 0) {
            // the first step's atoms were read by the caller ahead of the proposal
            const int j = lane, j2 = lane + kWave;
            candidate<NEW, OLD, CULL>(b, gg, j < n && j != skip, pre[0], px, py, pz, qx, qy, qz, acc, core, useful,
                                      qgas, ng);
            if (n > kWave)     // (a second block with no atom in it contributes nothing)
                candidate<NEW, OLD, CULL>(b, gg, j2 < n && j2 != skip, pre[1], px, py, pz, qx, qy, qz, acc, core,
                                          useful, qgas, ng);
            continue;
        }
        const int j = j0 + lane;
        const bool v1 = j < n;
        const Real4 ga = gas[v1 ? j : 0];
        if (U == 2) {
            const int j2 = j + kWave;
            const bool v2 = j2 < n;
            const Real4 gb = gas[v2 ? j2 : 0];
            candidate<NEW, OLD, CULL>(b, gg, v1 && j != skip, ga, px, py, pz, qx, qy, qz, acc, core, useful, qgas, ng);
            candidate<NEW, OLD, CULL>(b, gg, v2 && j2 != skip, gb, px, py, pz, qx, qy, qz, acc, core, useful, qgas,
                                      ng);
        } else {
            candidate<NEW, OLD, CULL>(b, gg, v1 && j != skip, ga, px, py, pz, qx, qy, qz, acc, core, useful, qgas, ng);
        }
    }
    const Real zmin = (NEW && OLD) ? (pz < qz ? pz : qz) : (NEW ? pz : qz);
    if (zmin < sv.top_plus_rc) {
        const bool bins = sv.bins != 0;
        const int total = bins ? 9 * sv.cap : sv.len;
        int cx = 0, cy = 0;
        if (bins) column_of(sv, OLD ? qx : px, OLD ? qy : py, cx, cy);
        // All U loads of a step are issued before the pair terms; entry kk of
        // the 9 * cap scanned is slot kk % cap of the block's column sp = kk / cap,
        // sp = 3 * (dy + 1) + (dx + 1).
        for (int k0 = part * U * kWave; k0 < total; k0 += STEP) {
            Real4 g[U];
            bool vv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = k0 + u * kWave + lane;
                vv[u] = k < total;
                const int kk = vv[u] ? k : 0;
                g[u] = sv.atoms[bins ? block_entry(sv, cx, cy, kk) : kk];
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                candidate<NEW, OLD, CULL>(b, gs, vv[u], g[u], px, py, pz, qx, qy, qz, acc, core, useful, qslab, ns);
        }
    }
    // (two waves per walker: the issue priority of the serial part of the trial, from
    // the wave reduction on; the sweep kernel lowered it for the pair loop)
    if (SPLIT == 2) __builtin_amdgcn_s_setprio(2);
    core_out = __any(core);
    if (CULL) {
        useful += lane == 0 ? (uint32_t)(ng + ns) : 0u;
        wave_sync();
        // LJ terms of the queued pairs: gas pairs, then slab pairs, in one lane space
        const int nq = ng + ns;
        for (int k0 = 0; k0 < nq; k0 += kWave) {
            const int k = k0 + lane;
            if (k < nq) {
                const bool is_gas = k < ng;
                const Real v = is_gas ? qgas[k] : qslab[k - ng];
                const Real r2 = v < Real(0) ? -v : v;
                const Real phi = lj_inside(r2, is_gas ? gg.sig2 : gs.sig2, is_gas ? gg.eps4 : gs.eps4,
                                           is_gas ? gg.shift : gs.shift);
                acc += v < Real(0) ? -phi : phi;
            }
        }
    }
    return wave_sum(acc);
}

}  // namespace fp64 / fp32
}  // namespace regc
