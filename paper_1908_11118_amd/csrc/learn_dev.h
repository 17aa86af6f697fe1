// learn_dev.h -- device-side definitions of the learned insertion proposal: the
// occupancy grid and network sizes, the sampler's copy of the network, the kernel
// arguments and LDS carve of the learned-proposal sampler, and the launchers shared
// by the sampler (learned.hip), the network code (mlp.hip) and the host runtime.
#pragma once
#include "regc_dev.h"

namespace regc {

// ---- learned insertion proposal ----
constexpr int kNetGrid = 16;                       // occupancy / proposal grid per axis
constexpr int kNetNV = kNetGrid * kNetGrid * kNetGrid;
constexpr int kNetH = 128;                         // hidden width

// The sampler's copy of the proposal network (bfloat16 weights, FP32 biases).
// W1 rows are the input voxels' weights ([4096][128]).  W2, W3 ([128 out][128 in])
// and W4 ([4096 out][128 in]) come in one of two layouts:
//  - k-major (the FP64 sampler, whose network arithmetic is sequential FP32 and
//    bit-reproducible): Wt[k][out];
//  - MFMA B-operand tiles (the FP32 sampler): for output tile t (16 outputs),
//    k-pair kp (32 inputs) and lane l, eight values
//      W[16 t + l % 16][32 kp + 16 (j / 4) + 4 (l / 16) + j % 4],  j = 0..7,
//    so one 16-byte load per lane feeds two 16x16x16 products.
struct NetDev {
    const uint16_t *w1, *w2, *w3, *w4;
    const float *b1, *b2, *b3, *b4;
};

constexpr int kMaxLearnClasses = 8;  // classes of a batch that can each carry a network

struct LearnArgs {
    NetDev net[kMaxLearnClasses];    // per class (entries of classes without a network unused)
    double alpha[kMaxLearnClasses];  // per class mixture weight of the network branch (0: uniform insertion)
    const int *walker_class;         // class of every walker
    const int *block_walker;         // walker of each workgroup (XCD-aware order)
    unsigned long long *evals;       // [0] network passes, [1] insertions served from the cached pass,
                                     // [2] network-branch insertions, [3] of them accepted
};

// LDS carve of the learned-proposal kernel (one walker per workgroup of kLearnWaves waves).
constexpr int kLearnWaves = 4;
struct LearnLds {
    size_t slab, lnk, xch, gas, vox, occ, list, part, hid, logit, bias, red, total;
};

__host__ __device__ inline LearnLds learn_lds(int max_slab_len, int gas_stride, int real_size)
{
    LearnLds L;
    const size_t r4 = 4 * (size_t)real_size;
    size_t off = 0;
    L.slab = off;    off = lds_round(off + (size_t)max_slab_len * r4);
    L.lnk = off;     off = lds_round(off + (size_t)(gas_stride + 2) * 8);
    L.xch = off;     off = lds_round(off + (size_t)2 * kLearnWaves * 2 * 8);
    L.gas = off;     off = lds_round(off + (size_t)gas_stride * r4);
    L.vox = off;     off = lds_round(off + (size_t)gas_stride * 4);
    L.occ = off;     off = lds_round(off + (size_t)kNetNV * 4);
    L.list = off;    off = lds_round(off + (size_t)(gas_stride + 1) * 4);
    L.part = off;    off = lds_round(off + (size_t)kLearnWaves * kNetH * 4);
    L.hid = off;     off = lds_round(off + (size_t)3 * kNetH * 2);
    L.logit = off;   off = lds_round(off + (size_t)kNetNV * 4);
    L.bias = off;    off = lds_round(off + (size_t)(kNetNV + 3 * kNetH) * 4);   // b4 | b1 | b2 | b3
    L.red = off;     off = lds_round(off + (size_t)kLearnWaves * 16 + 32);
    L.total = off;
    return L;
}

hipError_t launch_learned_f64(const SweepArgs &a, const LearnArgs &l, size_t smem, hipStream_t s);
hipError_t launch_learned_f32(const SweepArgs &a, const LearnArgs &l, size_t smem, hipStream_t s);
hipError_t launch_net_eval_f64(const NetDev &net, const ClassDev *cls, int cid, int stride, int n_conf,
                               const double *xyz, const int32_t *n, const int32_t *skip, float *logits, double *lse,
                               double *lnp, hipStream_t s);
hipError_t launch_net_eval_f32(const NetDev &net, const ClassDev *cls, int cid, int stride, int n_conf,
                               const double *xyz, const int32_t *n, const int32_t *skip, float *logits, double *lse,
                               double *lnp, hipStream_t s);

}  // namespace regc

struct regc_mlp;
namespace regc {
// Writes the sampler's copy of the network (layouts of NetDev: k-major when
// kmajor, else MFMA tiles) into caller-owned device buffers: w1 [4096*128],
// w2/w3 [128*128], w4 [4096*128] bfloat16 and the four bias vectors, on stream s.
// Returns a REGC_* code.
hipError_t launch_capture_voxels(int n_walkers, int stride, const ClassDev *cls, const int *walker_class,
                                 const int32_t *n, const double *xyz, int xyz_stride, uint16_t *vox, int32_t *n_out,
                                 hipStream_t s);
int mlp_export_sampler(regc_mlp *h, bool kmajor, uint16_t *w1, uint16_t *w2, uint16_t *w3, uint16_t *w4, float *b1,
                       float *b2, float *b3, float *b4, hipStream_t s);
}  // namespace regc
