// regc_dev.h -- data layouts shared by the HIP kernels and the host runtime of
// libregc_hip.so (internal; the public interface is include/regc.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace regc {

constexpr int kNStat = 10;
constexpr int kWave = 64;
constexpr int kMaxWalkersPerBlock = 8;

// Per-class constants (one class = one REGC simulation: slab, box, grid).
struct ClassDev {
    double lx, ly, zlo, zhi;
    double half_lx, half_ly, inv_lx, inv_ly;
    double lnv;              // ln V, V = lx * ly * (zhi - zlo)
    double slab_top;         // highest slab z (slab skipped above slab_top + rcut)
    int n_max;
    int trials;              // K trials per sweep
    int walker_off, n_walkers;   // global walkers [walker_off, walker_off + n_walkers)
    int state_off;           // global state index of this class's state 0 (== walker_off)
    int n_t, n_mu;
    // packed slab: entries [slab_off, slab_off + slab_len) of the slab arrays.
    // Without bins: the atoms in input order.  With bins: ncx*ncy columns of
    // `cap` entries each (padding entries sit at z = -1e4).
    int slab_off, slab_len;
    int bins;                // 0/1
    int ncx, ncy, cap;
    double inv_cw_x, inv_cw_y;
};

// Pair-potential constants, precomputed on the host.
struct PotDev {
    double sig2_gg, eps4_gg, shift_gg;
    double sig2_gs, eps4_gs, shift_gs;
    double rc2;
    double hc2_gg, hc2_gs;   // (hc_frac * sigma)^2
    int ideal;
};

struct SwapArgs {
    const ClassDev *cls;
    int32_t *label;
    int32_t *wos;                // [S_total] global walker holding global state
    const int32_t *n;
    const double *e;
    const double *beta, *lnz;
    uint32_t key0, key1;
    int64_t q;                   // exchange step index
    const int64_t *clock;        // if set: q = (clock[0] + interval) / swap_every - 1
    int interval, swap_every;
    int scheme;
    unsigned long long *att, *acc;   // [4][S_total]
    int S_total;
};

struct SweepArgs {
    const ClassDev *cls;
    const int *block_class;      // per block
    const int *block_w0;         // first global walker of the block
    const int *block_nw;         // walkers in the block
    const int *wslot;            // if set: the walker at block position block_w0 + slot
                                 // is wslot[block_w0 + slot] (a permutation within each class)
    int n_walkers;               // total walkers
    PotDev pot;
    int32_t *n;
    double *e;
    const int32_t *label;        // state index within the class
    double *xyz;                 // [W][xyz_stride][3]
    int xyz_stride;
    const double *beta, *lnz;    // [S_total]
    const double *lnk;           // log(k), k = 0 .. max n_max + 1
    const double *slab4;         // packed slab as double4 (FP64 kernels)
    const float *slab4f;         // packed slab as float4 (FP32 kernels)
    uint32_t key0, key1;
    uint64_t th_disp, th_ins;
    double max_disp;
    int64_t sweep0;
    const int64_t *clock;        // if set, the first sweep index is read from clock[0] (graph replays)
    int n_sweeps;
    int sample_every;
    int64_t rec_base;            // global record index of sample slot 0
    double *samp_e;
    int32_t *samp_n, *samp_s;
    unsigned long long *hist;    // [S_total][hist_stride]
    int hist_stride;
    unsigned long long *stats;   // [S_total][kNStat]
    unsigned long long *pairs;   // [0] candidate pairs evaluated, [1] of them inside the cutoff
    uint32_t *trace_bits;        // [trace sweep][W][trace_words] or null
    int32_t *trace_n;
    int64_t trace_sweep0, trace_cap;
    int trace_words;
    int max_slab_len;               // LDS carve sizes of this launch
    int gas_stride;                 // LDS entries per walker (max n_max over classes)
    int max_slab_scan;              // most slab candidates one trial scans (max over classes)
    int resync_every;               // > 0: running energy recomputed after every resync_every-th sweep
    int count_pairs;                // batched kernel: count the pair terms inside the cutoff
    // persistent launch: the exchange step inside the launch after every swap_every-th
    // sweep, between two grid-wide barriers (gbar: arrival count, generation; gerr set
    // when a barrier wait exceeded its bound)
    SwapArgs sw;
    int swap_every, n_class;
    unsigned int *gbar;
    int *gerr;
};

// Structural observables of every walker at a sample point (see regc.h).
struct ObsArgs {
    const ClassDev *cls;
    const int *walker_class;
    int n_walkers;
    const int32_t *n;
    const double *xyz;
    int xyz_stride;
    double dz, layer_lo, layer_hi, dr;
    int n_z, n_r, n_obs;
    uint32_t *out;               // [W][n_obs] of this record
};

// Lowest-energy recorded configuration per (class, N), updated at sample points.
struct MinArgs {
    const int *walker_class;
    int n_walkers, n_class, nN;  // nN = largest n_max + 1
    const int32_t *n;
    const double *e;
    const double *xyz;
    int xyz_stride;
    unsigned long long *key, *old_key;   // [n_class][nN] ordered energy bits (~0: none)
    int *widx;                           // [n_class][nN] INT_MAX between updates
    double *e_min;                       // [n_class][nN]
    double *xyz_min;                     // [n_class][nN][xyz_stride][3]
};

// The paper's REGC step (schedule 1): coin from Philox (0, step, 0xFFFFFFFF - class, 6).
struct PaperArgs {
    double x0;                   // probability of the particle-exchange attempt
    int mc_cycles;               // MC cycles of N displacements after each attempt
    // molecular dynamics as the canonical part (md_steps > 0 replaces the MC cycles)
    int md_steps;
    double md_dt, md_tau;        // time step (unit mass), thermostat time (0: none)
    double *vel;                 // [W][xyz_stride][3] velocities
    double *tv;                  // [W] temperature of the velocities (0: not drawn yet)
};

// LDS of the MD part after the sweep layout: per walker velocities and forces
// (double [gas_stride][3] each).
__host__ __device__ inline size_t md_lds_bytes(int gas_stride, int walkers)
{
    return (size_t)walkers * gas_stride * 48;
}


struct EnergyArgs {
    const ClassDev *cls;
    const int *walker_class;
    int n_walkers;
    PotDev pot;
    const int32_t *n;
    const double *xyz;
    int xyz_stride;
    const double *slab4;         // unbinned packed slab (double4), per class at unb_off
    const int *unb_off, *unb_len;
    double *e_out;
};

// LDS carve of the sweep kernel (byte offsets, 32-byte aligned), shared by the
// kernel and the host launch code: class slab, ln k table, the
// split-walker exchange slots, the walkers' gas coordinates, the pair queues.
struct LdsLayout {
    size_t slab, lnk, xch, gas, queue, total;
};

__host__ __device__ inline size_t lds_round(size_t x) { return (x + 31) & ~(size_t)31; }

__host__ __device__ inline LdsLayout lds_layout(int max_slab_len, int gas_stride, int max_slab_scan, int walkers,
                                                int queue_waves, int real_size)
{
    LdsLayout L;
    const size_t r4 = 4 * (size_t)real_size;
    size_t off = 0;
    L.slab = off;    off = lds_round(off + (size_t)max_slab_len * r4);
    L.lnk = off;     off = lds_round(off + (size_t)(gas_stride + 2) * 8);
    L.xch = off;     off = lds_round(off + (size_t)walkers * 16 * 8);
    L.gas = off;     off = lds_round(off + (size_t)walkers * gas_stride * r4);
    L.queue = off;   off = lds_round(off + (size_t)queue_waves * (2 * gas_stride + 2 * max_slab_scan) * real_size);
    L.total = off;
    return L;
}

// LDS carve of the batched-trial sweep kernel: class slab, ln k table, and per walker
// the gas coordinates and each particle's energy with the frozen slab.
struct BatchLds {
    size_t slab, lnk, gas, eslab, total;
};

__host__ __device__ inline BatchLds batch_lds(int max_slab_len, int gas_stride, int walkers, int real_size)
{
    BatchLds L;
    const size_t r4 = 4 * (size_t)real_size;
    size_t off = 0;
    L.slab = off;    off = lds_round(off + (size_t)max_slab_len * r4);
    L.lnk = off;     off = lds_round(off + (size_t)(gas_stride + 2) * 8);
    L.gas = off;     off = lds_round(off + (size_t)walkers * gas_stride * r4);
    L.eslab = off;   off = lds_round(off + (size_t)walkers * gas_stride * real_size);
    L.total = off;
    return L;
}

// LDS carve of the multi-wave batched-trial kernel (one walker per workgroup of B
// waves): class slab, ln k table, every wave's own copy of the gas coordinates and of
// each particle's energy with the frozen slab, and the double-buffered records the
// waves exchange after each pass (per wave: 8-byte outcome masks, 8 scenario energy
// changes, the slab energy at the new position).
struct MwLds {
    size_t slab, lnk, gas, eslab, rec, total;
};

constexpr int kMwRecDoubles = 10;

__host__ __device__ inline MwLds mw_lds(int max_slab_len, int gas_stride, int waves, int real_size)
{
    MwLds L;
    const size_t r4 = 4 * (size_t)real_size;
    size_t off = 0;
    L.slab = off;    off = lds_round(off + (size_t)max_slab_len * r4);
    L.lnk = off;     off = lds_round(off + (size_t)(gas_stride + 2) * 8);
    L.gas = off;     off = lds_round(off + (size_t)waves * gas_stride * r4);
    L.eslab = off;   off = lds_round(off + (size_t)waves * gas_stride * real_size);
    L.rec = off;     off = lds_round(off + (size_t)2 * waves * kMwRecDoubles * 8);
    L.total = off;
    return L;
}

// launchers (defined in the .hip files)
// batch: 2 or 4 runs a batched-trial kernel -- one wave per walker, or with split equal
// to batch one workgroup of `batch` waves per walker, one trial per wave -- else the
// one-trial kernel with `split` (1, 2 or 4) waves per walker and `cull`
hipError_t launch_sweep_f64(const SweepArgs &a, int n_blocks, int waves_per_block, int split, bool cull, int batch,
                            size_t smem, hipStream_t s);
hipError_t launch_sweep_f32(const SweepArgs &a, int n_blocks, int waves_per_block, int split, bool cull, int batch,
                            size_t smem, hipStream_t s);
// persistent form of the one-trial kernel (split 1 or 2, no cull): a cooperative launch
// of whole exchange intervals; fails when the grid cannot be resident at once
hipError_t launch_sweep_persist_f64(const SweepArgs &a, int n_blocks, int waves_per_block, int split, size_t smem,
                                    hipStream_t s);
hipError_t launch_sweep_persist_f32(const SweepArgs &a, int n_blocks, int waves_per_block, int split, size_t smem,
                                    hipStream_t s);
// workgroups of the persistent form that fit the device at once
hipError_t persist_capacity_f64(int waves_per_block, int split, size_t smem, int *max_blocks);
hipError_t persist_capacity_f32(int waves_per_block, int split, size_t smem, int *max_blocks);
hipError_t launch_paper_f64(const SweepArgs &a, const PaperArgs &p, int n_blocks, int waves_per_block, size_t smem,
                            hipStream_t s);
hipError_t launch_paper_f32(const SweepArgs &a, const PaperArgs &p, int n_blocks, int waves_per_block, size_t smem,
                            hipStream_t s);
hipError_t launch_swap(const SwapArgs &a, int n_class, hipStream_t s);
hipError_t launch_balance(const ClassDev *cls, int n_class, const int32_t *n, int wpb, int *wslot, hipStream_t s);
hipError_t launch_observables(const ObsArgs &a, hipStream_t s);
hipError_t launch_minima(const MinArgs &a, hipStream_t s);
hipError_t launch_clock_advance(int64_t *clock, int n, hipStream_t s);
hipError_t launch_clock_set(int64_t *clock, int64_t value, hipStream_t s);
hipError_t launch_energy_f64(const EnergyArgs &a, hipStream_t s);
hipError_t launch_energy_f32(const EnergyArgs &a, hipStream_t s);

}  // namespace regc
