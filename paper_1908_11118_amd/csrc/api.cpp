// api.cpp -- host runtime of libregc_hip.so: contexts, launch schedule of the
// sweep and exchange kernels, sample/trace/counter buffers, checkpointing.
// The public contract is include/regc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "host_util.h"
#include "learn_dev.h"

namespace regc {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

struct ClassHost {
    regc_system sys;
    std::vector<double> slab, t, mu;
    int S = 0, off = 0, K = 0;
    int bins = 0, ncx = 1, ncy = 1, cap = 0;
    std::vector<double> packed;   // xyz of the packed (binned or plain) slab, 3 per entry
};

struct TimingPair {
    hipEvent_t a, b;
};

}  // namespace regc

using namespace regc;

struct regc_ctx {
    regc_potential pot{};
    regc_opts opts{};
    std::vector<ClassHost> cls;
    int W = 0, nmax_all = 0, kmax = 0, words = 1;
    PotDev potd{};
    hipStream_t stream = nullptr;
    int wpb = 1, split = 1, nblocks = 0, max_slab_len = 0, max_slab_scan = 0;
    bool cull = false;
    bool balance = false;   // walker order by cost before each one-trial sweep launch
    int batch = 1;     // trials per pass of the sweep kernel (1: one-trial kernel)
    bool count_pairs = false;   // batched kernel: count pair terms inside the cutoff
    size_t smem = 0;

    DevBuf<ClassDev> cls_d;
    DevBuf<int> block_class_d, block_w0_d, block_nw_d, walker_class_d, unb_off_d, unb_len_d;
    DevBuf<int> wslot_d;       // walker order of the one-trial sweep launches (balance)
    DevBuf<int32_t> n_d, label_d, wos_d;
    DevBuf<double> e_d, xyz_d, beta_d, lnz_d, lnk_d, slab4_d, unb_d;
    DevBuf<float> slab4f_d;
    DevBuf<double> samp_e;
    DevBuf<int32_t> samp_n, samp_s;
    int64_t rec_cap = 0, rec_base = 0, n_rec = 0;
    DevBuf<unsigned long long> hist_d, stats_d, att_d, acc_d, pairs_d;
    DevBuf<uint32_t> trace_bits_d;
    DevBuf<int32_t> trace_n_d;
    int64_t trace_cap = 0, trace_sweep0 = 0;
    int64_t sweep = 0;
    std::vector<int> walker_class;

    bool timing = false;
    std::vector<TimingPair> ev_sweep, ev_swap;

    // molecular dynamics (paper schedule with md_steps > 0)
    DevBuf<double> vel_d, tv_d;

    // structural observables recorded with the samples
    bool obs_on = false;
    regc_observables obs_spec{};
    int obs_nz = 0, n_obs = 0;
    DevBuf<uint32_t> obs_d;             // [rec_cap][W][n_obs]
    // lowest-energy recorded configuration per (class, N)
    bool min_on = false;
    DevBuf<unsigned long long> minkey_d, minold_d;
    DevBuf<int> minw_d;
    DevBuf<double> mine_d, minxyz_d;

    // learned insertion proposal, per class (any alpha > 0: the learned kernel runs the sweeps);
    // net_w / net_b hold one network per class, allocated at the first proposal
    std::vector<double> alpha;
    DevBuf<int> learn_order_d;              // walker of each learned-kernel workgroup
    DevBuf<uint16_t> net_w;                 // w1 | w2p | w3p | w4p (bfloat16)
    DevBuf<float> net_b;                    // b1 | b2 | b3 | b4
    DevBuf<unsigned long long> net_ev_d;    // proposal counters [4]
    size_t learn_smem = 0;

    // graph replay of whole exchange intervals
    DevBuf<int64_t> clock_d;
    DevBuf<unsigned int> gbar_d;   // grid barrier of the persistent launch: arrivals, generation
    DevBuf<int> gerr_d;            // set when a grid barrier wait exceeded its bound
    bool persist_used = false;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;

    ~regc_ctx()
    {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        for (auto &p : ev_sweep) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
        for (auto &p : ev_swap) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
    }
};

// ---------------------------------------------------------------------------
extern "C" const char *regc_last_error(void) { return g_err; }

extern "C" const char *regc_strerror(int code)
{
    switch (code) {
    case REGC_OK: return "ok";
    case REGC_EINVAL: return "invalid argument";
    case REGC_ENOMEM: return "out of memory";
    case REGC_EHIP: return "HIP runtime error";
    case REGC_ECAPACITY: return "buffer capacity exceeded";
    case REGC_ESTATE: return "call made in the wrong order";
    case REGC_EUNSUPPORTED: return "unsupported option";
    case REGC_ENOCONV: return "reweighting did not converge";
    default: return "unknown error";
    }
}

extern "C" void regc_default_opts(regc_opts *o)
{
    std::memset(o, 0, sizeof *o);
    o->seed = 1;
    o->precision = REGC_FP64;
    o->p_disp = 0.5;
    o->p_ins = 0.25;
    o->max_disp = 0.2;
    o->trials_per_sweep = 0;
    o->swap_every = 10;
    o->sample_every = 1;
    o->swap_scheme = 0;
    o->sample_capacity = 0;
    o->trace_capacity = 0;
    o->walkers_per_block = 0;
    o->sweeps_per_launch = 0;
    o->slab_bins = 0;
    o->split = 0;
    o->cull = 0;
    o->graph_intervals = 0;
    o->schedule = 0;
    o->x0 = 0.99;
    o->mc_cycles = 10;
    o->md_steps = 0;
    o->md_dt = 0.005;
    o->md_tau = 0.1;
    o->resync_every = 0;
    o->batch_trials = 0;
    o->slab_cell = 0.0;
    o->persistent = 0;
    o->balance = 0;
}

static int validate(const regc_potential *pot, const regc_system *sys, const regc_grid *grid, const regc_opts *o)
{
    REGC_CHECK(pot && sys && grid && o, REGC_EINVAL, "null argument");
    REGC_CHECK(pot->mode == REGC_MODE_LJ || pot->mode == REGC_MODE_IDEAL, REGC_EUNSUPPORTED,
               "unsupported potential mode %d", pot->mode);
    REGC_CHECK(o->precision == REGC_FP64 || o->precision == REGC_FP32PAIR, REGC_EUNSUPPORTED,
               "unsupported precision %d", o->precision);
    REGC_CHECK(pot->rcut > 0 && pot->sig_gg > 0 && pot->sig_gs > 0 && pot->hc_frac >= 0, REGC_EINVAL,
               "rcut and sigmas must be positive");
    REGC_CHECK(grid->n_t > 0 && grid->n_mu > 0 && grid->t && grid->mu, REGC_EINVAL, "empty state grid");
    for (int l = 0; l < grid->n_t; ++l)
        REGC_CHECK(std::isfinite(grid->t[l]) && grid->t[l] > 0, REGC_EINVAL, "T must be positive and finite");
    for (int m = 0; m < grid->n_mu; ++m) REGC_CHECK(std::isfinite(grid->mu[m]), REGC_EINVAL, "mu must be finite");
    REGC_CHECK(sys->n_max >= 1 && sys->n_max <= 4095, REGC_EINVAL, "n_max must be in 1..4095");
    REGC_CHECK(sys->lx >= 2 * pot->rcut && sys->ly >= 2 * pot->rcut, REGC_EINVAL, "lx, ly must be >= 2 rcut");
    REGC_CHECK(sys->z_hi > sys->z_lo, REGC_EINVAL, "z_hi must exceed z_lo");
    REGC_CHECK(sys->lambda1 > 0, REGC_EINVAL, "lambda1 must be positive");
    REGC_CHECK(sys->n_slab >= 0 && (sys->n_slab == 0 || sys->slab_xyz), REGC_EINVAL, "slab coordinates missing");
    REGC_CHECK(o->p_disp >= 0 && o->p_ins >= 0 && o->p_disp + o->p_ins <= 1.0, REGC_EINVAL, "bad move mix");
    REGC_CHECK(std::fabs(o->p_ins - (1.0 - o->p_disp - o->p_ins)) < 1e-12, REGC_EINVAL,
               "insertion and removal probabilities must be equal");
    REGC_CHECK(o->max_disp >= 0 && o->max_disp < 0.5 * std::min(sys->lx, sys->ly), REGC_EINVAL, "bad max_disp");
    REGC_CHECK(o->swap_every >= 0 && o->sample_every >= 0 && o->trials_per_sweep >= 0, REGC_EINVAL,
               "negative schedule value");
    REGC_CHECK(o->swap_scheme == 0 || o->swap_scheme == 1, REGC_EUNSUPPORTED, "unknown swap scheme");
    REGC_CHECK(o->walkers_per_block >= 0 && o->walkers_per_block <= kMaxWalkersPerBlock, REGC_EINVAL,
               "walkers_per_block must be 0..%d", kMaxWalkersPerBlock);
    REGC_CHECK(o->split >= 0 && o->split <= 4 && o->split != 3, REGC_EINVAL, "split must be 0, 1, 2 or 4");
    REGC_CHECK(o->graph_intervals >= 0 && o->graph_intervals <= 1000, REGC_EINVAL, "graph_intervals must be 0..1000");
    REGC_CHECK(o->schedule == 0 || o->schedule == 1, REGC_EUNSUPPORTED, "unknown schedule %d", o->schedule);
    REGC_CHECK(o->resync_every >= -1, REGC_EINVAL, "resync_every must be -1, 0 or positive");
    REGC_CHECK(o->slab_cell == 0.0 || (o->slab_cell >= 1.0 && o->slab_cell <= 16.0), REGC_EINVAL,
               "slab_cell must be 0 or in [1, 16]");
    REGC_CHECK(o->persistent >= 0, REGC_EINVAL, "persistent must be 0 or positive");
    REGC_CHECK(o->balance >= -1 && o->balance <= 1, REGC_EINVAL, "balance must be -1, 0 or 1");
    REGC_CHECK(o->persistent == 0 || (o->schedule == 0 && o->graph_intervals == 0 && o->batch_trials <= 1 &&
                                      o->cull <= 0 && o->split <= 2 && o->swap_every > 0),
               REGC_EINVAL, "persistent launches need the sweep schedule with exchanges, one trial at a time, "
                            "split 0, 1 or 2, no cull and no graph replay");
    REGC_CHECK(o->batch_trials >= 0 && o->batch_trials <= 4 && o->batch_trials != 3, REGC_EINVAL,
               "batch_trials must be 0, 1, 2 or 4");
    if (o->schedule == 1) {
        REGC_CHECK(o->x0 >= 0.0 && o->x0 <= 1.0, REGC_EINVAL, "x0 must lie in [0, 1]");
        REGC_CHECK(o->mc_cycles >= 0 && o->mc_cycles <= 1000, REGC_EINVAL, "mc_cycles must be 0..1000");
        REGC_CHECK(o->graph_intervals == 0, REGC_EUNSUPPORTED, "the paper schedule has no graph replay");
        REGC_CHECK(o->md_steps >= 0 && o->md_steps <= 100000 && o->md_dt > 0 && o->md_tau >= 0, REGC_EINVAL,
                   "bad molecular-dynamics parameters");
    }
    return REGC_OK;
}

static void pack_slab(ClassHost &c, const regc_potential *pot, const regc_opts *o)
{
    const int ns = c.sys.n_slab;
    const double lx = c.sys.lx, ly = c.sys.ly;
    const double cw = (pot->rcut + o->max_disp) * (o->slab_cell > 1.0 ? o->slab_cell : 1.0);
    const int ncx = (int)std::floor(lx / cw);
    const int ncy = (int)std::floor(ly / cw);
    const bool bins = ns > 0 && ncx >= 3 && ncy >= 3 && o->slab_bins >= 0;
    c.bins = bins ? 1 : 0;
    c.packed.clear();
    if (!bins) {
        c.ncx = c.ncy = 1;
        c.cap = ns;
        c.packed = c.slab;
        return;
    }
    c.ncx = ncx;
    c.ncy = ncy;
    const double cwx = lx / ncx, cwy = ly / ncy;
    std::vector<std::vector<int>> col(ncx * ncy);
    for (int a = 0; a < ns; ++a) {
        double x = std::fmod(c.slab[3 * a], lx), y = std::fmod(c.slab[3 * a + 1], ly);
        if (x < 0) x += lx;
        if (y < 0) y += ly;
        int cx = std::min(ncx - 1, std::max(0, (int)(x / cwx)));
        int cy = std::min(ncy - 1, std::max(0, (int)(y / cwy)));
        col[cy * ncx + cx].push_back(a);
    }
    int cap = 1;
    for (auto &v : col) cap = std::max(cap, (int)v.size());
    c.cap = cap;
    c.packed.assign((size_t)ncx * ncy * cap * 3, 0.0);
    for (int k = 0; k < ncx * ncy; ++k)
        for (int j = 0; j < cap; ++j) {
            double *d = &c.packed[((size_t)k * cap + j) * 3];
            if (j < (int)col[k].size()) {
                const int a = col[k][j];
                d[0] = c.slab[3 * a]; d[1] = c.slab[3 * a + 1]; d[2] = c.slab[3 * a + 2];
            } else {
                d[0] = 0.0; d[1] = 0.0; d[2] = -1.0e4;   // padding, beyond any cutoff
            }
        }
}

static int upload(void *dst, const void *src, size_t bytes)
{
    if (bytes == 0) return REGC_OK;
    REGC_HIP(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
    return REGC_OK;
}

static int ctx_alloc_and_init(regc_ctx *c)
{
    const regc_opts &o = c->opts;
    int rc;
    int W = 0, kmax = 0, nmax = 0, n_class = (int)c->cls.size();
    for (auto &k : c->cls) {
        k.off = W;
        k.S = (int)(k.t.size() * k.mu.size());
        k.K = o.schedule == 1 ? 1 + o.mc_cycles * k.sys.n_max
                              : (o.trials_per_sweep > 0 ? o.trials_per_sweep : k.sys.n_max + 1);
        W += k.S;
        kmax = std::max(kmax, k.K);
        nmax = std::max(nmax, k.sys.n_max);
        pack_slab(k, &c->pot, &o);
    }
    c->W = W;
    c->kmax = kmax;
    c->nmax_all = nmax;
    c->words = (kmax + 31) / 32;

    // potential constants (same arithmetic order as the definitions in regc.h)
    const regc_potential &p = c->pot;
    PotDev &pd = c->potd;
    auto shift = [&](double eps, double sig) {
        if (!p.shifted) return 0.0;
        const double c2 = (sig * sig) / (p.rcut * p.rcut);
        const double c6 = c2 * c2 * c2;
        return 4.0 * eps * (c6 * c6 - c6);
    };
    pd.sig2_gg = p.sig_gg * p.sig_gg; pd.eps4_gg = 4.0 * p.eps_gg; pd.shift_gg = shift(p.eps_gg, p.sig_gg);
    pd.sig2_gs = p.sig_gs * p.sig_gs; pd.eps4_gs = 4.0 * p.eps_gs; pd.shift_gs = shift(p.eps_gs, p.sig_gs);
    pd.rc2 = p.rcut * p.rcut;
    pd.hc2_gg = (p.hc_frac * p.sig_gg) * (p.hc_frac * p.sig_gg);
    pd.hc2_gs = (p.hc_frac * p.sig_gs) * (p.hc_frac * p.sig_gs);
    pd.ideal = p.mode == REGC_MODE_IDEAL;

    // per-class device constants, packed slabs
    std::vector<ClassDev> cd(n_class);
    std::vector<double> slab4, unb4;
    std::vector<float> slab4f;
    std::vector<int> unb_off(n_class), unb_len(n_class);
    int max_slab_len = 0;
    for (int k = 0; k < n_class; ++k) {
        ClassHost &h = c->cls[k];
        ClassDev &d = cd[k];
        d.lx = h.sys.lx; d.ly = h.sys.ly; d.zlo = h.sys.z_lo; d.zhi = h.sys.z_hi;
        d.half_lx = 0.5 * h.sys.lx; d.half_ly = 0.5 * h.sys.ly;
        d.inv_lx = 1.0 / h.sys.lx; d.inv_ly = 1.0 / h.sys.ly;
        d.lnv = std::log(h.sys.lx * h.sys.ly * (h.sys.z_hi - h.sys.z_lo));
        double top = -1.0e30;
        for (int a = 0; a < h.sys.n_slab; ++a) top = std::max(top, h.slab[3 * a + 2]);
        d.slab_top = top;
        d.n_max = h.sys.n_max;
        d.trials = h.K;
        d.walker_off = h.off; d.n_walkers = h.S; d.state_off = h.off;
        d.n_t = (int)h.t.size(); d.n_mu = (int)h.mu.size();
        const int len = (int)(h.packed.size() / 3);
        d.slab_off = (int)(slab4.size() / 4);
        d.slab_len = len;
        for (int j = 0; j < len; ++j) {
            for (int q = 0; q < 3; ++q) { slab4.push_back(h.packed[3 * j + q]); slab4f.push_back((float)h.packed[3 * j + q]); }
            slab4.push_back(0.0);
            slab4f.push_back(0.f);
        }
        unb_off[k] = (int)(unb4.size() / 4);
        unb_len[k] = h.sys.n_slab;
        for (int j = 0; j < h.sys.n_slab; ++j) {
            for (int q = 0; q < 3; ++q) unb4.push_back(h.slab[3 * j + q]);
            unb4.push_back(0.0);
        }
        d.bins = h.bins; d.ncx = h.ncx; d.ncy = h.ncy; d.cap = h.cap;
        d.inv_cw_x = h.bins ? h.ncx / h.sys.lx : 0.0;
        d.inv_cw_y = h.bins ? h.ncy / h.sys.ly : 0.0;
        max_slab_len = std::max(max_slab_len, len);
        c->max_slab_scan = std::max(c->max_slab_scan, h.bins ? 9 * h.cap : len);
    }
    c->max_slab_len = max_slab_len;

    // launch shape: walkers per block, waves per walker, LDS
    int dev = 0;
    REGC_HIP(hipGetDevice(&dev));
    int lds_max = 0, n_cu = 0, lds_cu = 0;
    REGC_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    REGC_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    REGC_HIP(hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev));
    if (lds_cu <= 0) lds_cu = lds_max;
    const int real = o.precision == REGC_FP64 ? 8 : 4;
    // waves per walker unless asked: two while one each would leave at most one wave
    // per SIMD (W <= 4 x CUs: a walker's trial chain is latency-bound and the second
    // wave halves its pair loop; measured 2.8 % faster at 1024 walkers and 2.2 % at 64
    // on 256 CUs), one above that (25 % slower with two at 4096 walkers, where four
    // walkers per SIMD already hide the latency).  The paper's step keeps one.
    // one trial at a time unless batched trials are requested (measured slower at 1024
    // walkers on 256 CUs: one wave per SIMD leaves the batch's serial decisions exposed)
    const int batch = o.schedule != 0 ? 1 : (o.batch_trials > 0 ? o.batch_trials : 1);
    // batched trials with split equal to the batch: one wave per trial (the multi-wave form)
    int split = batch > 1 ? (o.split == batch ? batch : 1)
                          : (o.split > 0 ? o.split
                                         : ((o.schedule == 0 && o.walkers_per_block == 0 && W <= 4 * n_cu &&
                                             c->pot.mode != REGC_MODE_IDEAL) ? 2 : 1));
    const bool cull = batch == 1 && o.cull > 0;
    auto smem_for = [&](int wpb) {
        if (batch > 1 && split == batch) return mw_lds(max_slab_len, nmax, batch, real).total;
        if (batch > 1) return batch_lds(max_slab_len, nmax, wpb, real).total;
        return lds_layout(max_slab_len, nmax, c->max_slab_scan, wpb, cull ? wpb * split : 0, real).total;
    };
    int wpb = split > 1 ? 1 : o.walkers_per_block;
    if (wpb == 0) {
        wpb = 1;
        if (W >= 1024) {
            // the walkers a compute unit must hold (at most four waves per SIMD), and the
            // workgroup size that lets its LDS hold them all: 4 walkers per workgroup, or 8
            // when a workgroup of 4 leaves too little LDS for the rest (each workgroup
            // carries its own slab and ln k copies; measured 1.36e9 against 1.12e9 trial
            // moves/s for the 4096-replica uneven batch, whose four-walker workgroups of
            // 500-atom walkers fit three to a compute unit)
            const int need = std::min(16, (W + n_cu - 1) / n_cu);
            auto resident = [&](int k) {
                const size_t b = smem_for(k);
                if (b > (size_t)lds_max) return 0;
                return std::min(need, (int)(lds_cu / b) * k);
            };
            wpb = resident(8) > resident(4) ? 8 : 4;
        }
    }
    while (wpb > 1 && smem_for(wpb) > (size_t)lds_max) --wpb;
    REGC_CHECK(smem_for(wpb) <= (size_t)lds_max, REGC_EUNSUPPORTED,
               "one walker needs %zu bytes of LDS, the device allows %d", smem_for(wpb), lds_max);
    c->wpb = wpb;
    c->split = split;
    c->cull = cull;
    // walker order by cost: on by default where several walkers share a SIMD (the
    // SIMDs' throughput is the limit, and neighbouring states with similar particle
    // counts in one workgroup left compute units idle while others ran: 4096-replica
    // uneven batch 14.9 -> 11.6 ms per launch), off at one walker per SIMD, where each
    // chain's latency is the limit and the extra launch only costs (1 %, 1024 walkers)
    c->balance = o.balance > 0 || (o.balance == 0 && W > 4 * n_cu);
    c->batch = batch;
    c->smem = smem_for(wpb);
    if (o.schedule == 1 && o.md_steps > 0) {
        c->smem = lds_round(c->smem) + md_lds_bytes(nmax, wpb);
        REGC_CHECK(c->smem <= (size_t)lds_max, REGC_EUNSUPPORTED, "molecular dynamics needs %zu bytes of LDS",
                   c->smem);
    }
    std::vector<int> bcls, bw0, bnw;
    c->walker_class.assign(W, 0);
    // blocks of the costliest classes first (largest n_max + slab candidates), so the
    // long-running walkers start early and the launch ends with the short ones
    std::vector<int> order(n_class);
    for (int k = 0; k < n_class; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const ClassHost &ha = c->cls[a], &hb = c->cls[b];
        return ha.sys.n_max + (ha.bins ? 9 * ha.cap : (int)(ha.packed.size() / 3)) >
               hb.sys.n_max + (hb.bins ? 9 * hb.cap : (int)(hb.packed.size() / 3));
    });
    for (int k : order) {
        const ClassHost &h = c->cls[k];
        for (int w = 0; w < h.S; w += wpb) {
            bcls.push_back(k);
            bw0.push_back(h.off + w);
            bnw.push_back(std::min(wpb, h.S - w));
        }
        for (int w = 0; w < h.S; ++w) c->walker_class[h.off + w] = k;
    }
    c->nblocks = (int)bcls.size();

    // state constants: ln z = beta mu - 3 ln(lambda1 / sqrt(T))
    std::vector<double> beta(W), lnz(W);
    std::vector<int32_t> label(W), wos(W);
    for (auto &h : c->cls) {
        const int M = (int)h.mu.size();
        for (int l = 0; l < (int)h.t.size(); ++l)
            for (int m = 0; m < M; ++m) {
                const double T = h.t[l];
                const double b = 1.0 / T;
                beta[h.off + l * M + m] = b;
                lnz[h.off + l * M + m] = b * h.mu[m] - 3.0 * std::log(h.sys.lambda1 / std::sqrt(T));
            }
        for (int w = 0; w < h.S; ++w) { label[h.off + w] = w; wos[h.off + w] = h.off + w; }
    }
    std::vector<double> lnk(nmax + 2);
    lnk[0] = 0.0;
    for (int k = 1; k <= nmax + 1; ++k) lnk[k] = std::log((double)k);

    const int64_t rec_cap = o.sample_every > 0 ? std::max<int64_t>(1, o.sample_capacity > 0 ? o.sample_capacity / W : 1024) : 0;
    c->rec_cap = rec_cap;
    c->trace_cap = o.trace_capacity;

    if ((rc = c->cls_d.alloc(n_class)) || (rc = c->block_class_d.alloc(c->nblocks)) ||
        (rc = c->block_w0_d.alloc(c->nblocks)) || (rc = c->block_nw_d.alloc(c->nblocks)) ||
        (rc = c->walker_class_d.alloc(W)) || (rc = c->unb_off_d.alloc(n_class)) || (rc = c->unb_len_d.alloc(n_class)) ||
        (rc = c->n_d.alloc(W)) || (rc = c->label_d.alloc(W)) || (rc = c->wos_d.alloc(W)) || (rc = c->e_d.alloc(W)) ||
        (rc = c->xyz_d.alloc((size_t)W * nmax * 3)) || (rc = c->beta_d.alloc(W)) || (rc = c->lnz_d.alloc(W)) ||
        (rc = c->lnk_d.alloc(nmax + 2)) || (rc = c->slab4_d.alloc(slab4.size())) ||
        (rc = c->slab4f_d.alloc(slab4f.size())) || (rc = c->unb_d.alloc(unb4.size())) ||
        (rc = c->samp_e.alloc((size_t)rec_cap * W)) ||
        (rc = c->samp_n.alloc((size_t)rec_cap * W)) || (rc = c->samp_s.alloc((size_t)rec_cap * W)) ||
        (rc = c->hist_d.alloc((size_t)W * (nmax + 1))) || (rc = c->stats_d.alloc((size_t)W * kNStat)) ||
        (rc = c->att_d.alloc((size_t)4 * W)) || (rc = c->acc_d.alloc((size_t)4 * W)) || (rc = c->pairs_d.alloc(2)) ||
        (rc = c->trace_bits_d.alloc((size_t)std::max<int64_t>(c->trace_cap, 0) * W * c->words)) ||
        (rc = c->trace_n_d.alloc((size_t)std::max<int64_t>(c->trace_cap, 0) * W)) || (rc = c->clock_d.alloc(1)) ||
        (rc = c->gbar_d.alloc(2)) || (rc = c->gerr_d.alloc(1)) || (rc = c->wslot_d.alloc(W)))
        return rc;
    REGC_HIP(hipMemset(c->gbar_d.p, 0, sizeof(unsigned int) * 2));
    REGC_HIP(hipMemset(c->gerr_d.p, 0, sizeof(int)));
    if (o.schedule == 1 && o.md_steps > 0) {
        if ((rc = c->vel_d.alloc((size_t)W * nmax * 3)) || (rc = c->tv_d.alloc(W))) return rc;
        REGC_HIP(hipMemset(c->vel_d.p, 0, sizeof(double) * (size_t)W * nmax * 3));
        REGC_HIP(hipMemset(c->tv_d.p, 0, sizeof(double) * W));
    }
    if ((rc = upload(c->cls_d.p, cd.data(), sizeof(ClassDev) * n_class)) ||
        (rc = upload(c->block_class_d.p, bcls.data(), sizeof(int) * bcls.size())) ||
        (rc = upload(c->block_w0_d.p, bw0.data(), sizeof(int) * bw0.size())) ||
        (rc = upload(c->block_nw_d.p, bnw.data(), sizeof(int) * bnw.size())) ||
        (rc = upload(c->walker_class_d.p, c->walker_class.data(), sizeof(int) * W)) ||
        (rc = upload(c->unb_off_d.p, unb_off.data(), sizeof(int) * n_class)) ||
        (rc = upload(c->unb_len_d.p, unb_len.data(), sizeof(int) * n_class)) ||
        (rc = upload(c->label_d.p, label.data(), sizeof(int32_t) * W)) ||
        (rc = upload(c->wos_d.p, wos.data(), sizeof(int32_t) * W)) ||
        (rc = upload(c->beta_d.p, beta.data(), sizeof(double) * W)) ||
        (rc = upload(c->lnz_d.p, lnz.data(), sizeof(double) * W)) ||
        (rc = upload(c->lnk_d.p, lnk.data(), sizeof(double) * lnk.size())) ||
        (rc = upload(c->slab4_d.p, slab4.data(), sizeof(double) * slab4.size())) ||
        (rc = upload(c->slab4f_d.p, slab4f.data(), sizeof(float) * slab4f.size())) ||
        (rc = upload(c->unb_d.p, unb4.data(), sizeof(double) * unb4.size())))
        return rc;
    REGC_HIP(hipMemset(c->n_d.p, 0, sizeof(int32_t) * W));
    REGC_HIP(hipMemset(c->e_d.p, 0, sizeof(double) * W));
    REGC_HIP(hipMemset(c->xyz_d.p, 0, sizeof(double) * (size_t)W * nmax * 3));
    REGC_HIP(hipMemset(c->hist_d.p, 0, sizeof(unsigned long long) * (size_t)W * (nmax + 1)));
    REGC_HIP(hipMemset(c->stats_d.p, 0, sizeof(unsigned long long) * (size_t)W * kNStat));
    REGC_HIP(hipMemset(c->att_d.p, 0, sizeof(unsigned long long) * 4 * W));
    REGC_HIP(hipMemset(c->acc_d.p, 0, sizeof(unsigned long long) * 4 * W));
    REGC_HIP(hipMemset(c->pairs_d.p, 0, sizeof(unsigned long long) * 2));
    REGC_HIP(hipDeviceSynchronize());
    return REGC_OK;
}

static int create_common(int n_class, const regc_potential *pot, const regc_system *sys, const regc_grid *grid,
                         const regc_opts *opts, regc_ctx **out)
{
    REGC_CHECK(out, REGC_EINVAL, "null output pointer");
    REGC_CHECK(n_class >= 1, REGC_EINVAL, "need at least one class");
    REGC_CHECK(!opts || opts->schedule != 1 || n_class == 1, REGC_EUNSUPPORTED,
               "the paper schedule runs single-class contexts");
    *out = nullptr;
    for (int k = 0; k < n_class; ++k) {
        int rc = validate(pot, sys + k, grid + k, opts);
        if (rc) return rc;
    }
    regc_ctx *c = new regc_ctx();
    c->pot = *pot;
    c->opts = *opts;
    for (int k = 0; k < n_class; ++k) {
        ClassHost h;
        h.sys = sys[k];
        h.slab.assign(sys[k].slab_xyz, sys[k].slab_xyz + 3 * (size_t)sys[k].n_slab);
        h.sys.slab_xyz = nullptr;
        h.t.assign(grid[k].t, grid[k].t + grid[k].n_t);
        h.mu.assign(grid[k].mu, grid[k].mu + grid[k].n_mu);
        c->cls.push_back(std::move(h));
    }
    int rc = ctx_alloc_and_init(c);
    if (rc) {
        delete c;
        return rc;
    }
    *out = c;
    return REGC_OK;
}

extern "C" int regc_create(const regc_potential *pot, const regc_system *sys, const regc_grid *grid,
                           const regc_opts *opts, regc_ctx **out)
{
    return create_common(1, pot, sys, grid, opts, out);
}

extern "C" int regc_create_batch(int n_class, const regc_potential *pot, const regc_system *sys,
                                 const regc_grid *grid, const regc_opts *opts, regc_ctx **out)
{
    REGC_CHECK(sys && grid, REGC_EINVAL, "null argument");
    return create_common(n_class, pot, sys, grid, opts, out);
}

extern "C" int regc_get_layout(const regc_ctx *c, int *n_class, int *offsets, int *counts)
{
    REGC_CHECK(c, REGC_EINVAL, "null context");
    if (n_class) *n_class = (int)c->cls.size();
    for (size_t k = 0; k < c->cls.size(); ++k) {
        if (offsets) offsets[k] = c->cls[k].off;
        if (counts) counts[k] = c->cls[k].S;
    }
    return REGC_OK;
}

extern "C" int regc_set_stream(regc_ctx *c, void *stream)
{
    REGC_CHECK(c, REGC_EINVAL, "null context");
    c->stream = (hipStream_t)stream;
    return REGC_OK;
}

static int record_event(regc_ctx *c, std::vector<TimingPair> &v, bool start)
{
    if (start) {
        TimingPair p;
        REGC_HIP(hipEventCreate(&p.a));
        REGC_HIP(hipEventCreate(&p.b));
        REGC_HIP(hipEventRecord(p.a, c->stream));
        v.push_back(p);
    } else {
        REGC_HIP(hipEventRecord(v.back().b, c->stream));
    }
    return REGC_OK;
}

// Weights and biases of one proposal network in the sampler's layout.
static constexpr size_t kNetWords = 2 * (size_t)kNetNV * kNetH + 2 * (size_t)kNetH * kNetH;
static constexpr size_t kNetBiases = 3 * (size_t)kNetH + kNetNV;

static bool learned_on(const regc_ctx *c)
{
    for (double a : c->alpha)
        if (a > 0.0) return true;
    return false;
}

static SweepArgs sweep_args(regc_ctx *c, int64_t sweep0, int n, bool use_clock)
{
    SweepArgs a{};
    a.cls = c->cls_d.p;
    a.block_class = c->block_class_d.p;
    a.block_w0 = c->block_w0_d.p;
    a.block_nw = c->block_nw_d.p;
    a.n_walkers = c->W;
    a.pot = c->potd;
    a.n = c->n_d.p;
    a.e = c->e_d.p;
    a.label = c->label_d.p;
    a.xyz = c->xyz_d.p;
    a.xyz_stride = c->nmax_all;
    a.beta = c->beta_d.p;
    a.lnz = c->lnz_d.p;
    a.lnk = c->lnk_d.p;
    a.slab4 = c->slab4_d.p;
    a.slab4f = c->slab4f_d.p;
    a.key0 = (uint32_t)c->opts.seed;
    a.key1 = (uint32_t)(c->opts.seed >> 32);
    a.th_disp = (uint64_t)std::llround(c->opts.p_disp * 4294967296.0);
    a.th_ins = a.th_disp + (uint64_t)std::llround(c->opts.p_ins * 4294967296.0);
    a.max_disp = c->opts.max_disp;
    a.sweep0 = sweep0;              // with the clock: offset from clock[0]
    a.clock = use_clock ? c->clock_d.p : nullptr;
    a.n_sweeps = n;
    a.sample_every = c->opts.sample_every;
    a.rec_base = c->rec_base;
    a.samp_e = c->samp_e.p;
    a.samp_n = c->samp_n.p;
    a.samp_s = c->samp_s.p;
    a.hist = c->hist_d.p;
    a.hist_stride = c->nmax_all + 1;
    a.stats = c->stats_d.p;
    a.pairs = c->pairs_d.p;
    a.trace_bits = c->trace_cap > 0 ? c->trace_bits_d.p : nullptr;
    a.trace_n = c->trace_cap > 0 ? c->trace_n_d.p : nullptr;
    a.trace_sweep0 = c->trace_sweep0;
    a.trace_cap = c->trace_cap;
    a.trace_words = c->words;
    a.max_slab_len = c->max_slab_len;
    a.gas_stride = c->nmax_all;
    a.max_slab_scan = c->max_slab_scan;
    a.count_pairs = c->count_pairs ? 1 : 0;
    a.resync_every = c->opts.resync_every > 0 ? c->opts.resync_every
                                              : (c->opts.resync_every == 0 && c->opts.precision == REGC_FP32PAIR ? 100 : 0);
    return a;
}

static int launch_sweeps(regc_ctx *c, int64_t sweep0, int n, hipStream_t stream, bool use_clock)
{
    SweepArgs a = sweep_args(c, sweep0, n, use_clock);
    int rc;
    const bool ev = c->timing && !use_clock;
    if (ev && (rc = record_event(c, c->ev_sweep, true))) return rc;
    if (c->opts.schedule == 1) {
        PaperArgs pa{};
        pa.x0 = c->opts.x0;
        pa.mc_cycles = c->opts.mc_cycles;
        pa.md_steps = c->opts.md_steps;
        pa.md_dt = c->opts.md_dt;
        pa.md_tau = c->opts.md_tau;
        pa.vel = c->vel_d.p;
        pa.tv = c->tv_d.p;
        if (c->opts.precision == REGC_FP64)
            REGC_HIP(launch_paper_f64(a, pa, c->nblocks, c->wpb, c->smem, stream));
        else
            REGC_HIP(launch_paper_f32(a, pa, c->nblocks, c->wpb, c->smem, stream));
    } else if (learned_on(c)) {
        LearnArgs l{};
        for (size_t k = 0; k < c->cls.size(); ++k) {
            l.alpha[k] = c->alpha[k];
            if (c->alpha[k] == 0.0) continue;
            const uint16_t *w = c->net_w.p + k * kNetWords;
            const float *bb = c->net_b.p + k * kNetBiases;
            NetDev &d = l.net[k];
            d.w1 = w;
            d.w2 = w + (size_t)kNetNV * kNetH;
            d.w3 = d.w2 + (size_t)kNetH * kNetH;
            d.w4 = d.w3 + (size_t)kNetH * kNetH;
            d.b1 = bb;
            d.b2 = bb + kNetH;
            d.b3 = bb + 2 * kNetH;
            d.b4 = bb + 3 * kNetH;
        }
        l.walker_class = c->walker_class_d.p;
        l.block_walker = c->learn_order_d.p;
        l.evals = c->net_ev_d.p;
        if (c->opts.precision == REGC_FP64)
            REGC_HIP(launch_learned_f64(a, l, c->learn_smem, stream));
        else
            REGC_HIP(launch_learned_f32(a, l, c->learn_smem, stream));
    } else {
        if (c->batch == 1 && c->balance) {
            REGC_HIP(launch_balance(c->cls_d.p, (int)c->cls.size(), c->n_d.p, c->wpb, c->wslot_d.p, stream));
            a.wslot = c->wslot_d.p;
        }
        if (c->opts.precision == REGC_FP64)
            REGC_HIP(launch_sweep_f64(a, c->nblocks, c->wpb * c->split, c->split, c->cull, c->batch, c->smem, stream));
        else
            REGC_HIP(launch_sweep_f32(a, c->nblocks, c->wpb * c->split, c->split, c->cull, c->batch, c->smem, stream));
    }
    if (ev && (rc = record_event(c, c->ev_sweep, false))) return rc;
    return REGC_OK;
}

static SwapArgs swap_args(regc_ctx *c, int64_t q, bool use_clock)
{
    SwapArgs a{};
    a.cls = c->cls_d.p;
    a.label = c->label_d.p;
    a.wos = c->wos_d.p;
    a.n = c->n_d.p;
    a.e = c->e_d.p;
    a.beta = c->beta_d.p;
    a.lnz = c->lnz_d.p;
    a.key0 = (uint32_t)c->opts.seed;
    a.key1 = (uint32_t)(c->opts.seed >> 32);
    a.q = q;
    a.scheme = c->opts.swap_scheme;
    a.att = c->att_d.p;
    a.acc = c->acc_d.p;
    a.S_total = c->W;
    a.clock = use_clock ? c->clock_d.p : nullptr;
    a.interval = c->opts.swap_every;
    a.swap_every = c->opts.swap_every;
    return a;
}

static int launch_exchange(regc_ctx *c, int64_t q, hipStream_t stream, bool use_clock)
{
    SwapArgs a = swap_args(c, q, use_clock);
    int rc;
    const bool ev = c->timing && !use_clock;
    if (ev && (rc = record_event(c, c->ev_swap, true))) return rc;
    REGC_HIP(launch_swap(a, (int)c->cls.size(), stream));
    if (ev && (rc = record_event(c, c->ev_swap, false))) return rc;
    return REGC_OK;
}

// `intervals` whole exchange intervals from sweep0 (an interval boundary) in one
// cooperative launch of the persistent sweep kernel, the exchange steps inside it.
static int launch_persistent(regc_ctx *c, int64_t sweep0, int intervals)
{
    const int se = c->opts.swap_every;
    SweepArgs a = sweep_args(c, sweep0, intervals * se, false);
    a.sw = swap_args(c, 0, false);
    a.swap_every = se;
    a.n_class = (int)c->cls.size();
    a.gbar = c->gbar_d.p;
    a.gerr = c->gerr_d.p;
    int max_blocks = 0;
    const int wpb_waves = c->wpb * c->split;
    if (c->opts.precision == REGC_FP64)
        REGC_HIP(persist_capacity_f64(wpb_waves, c->split, c->smem, &max_blocks));
    else
        REGC_HIP(persist_capacity_f32(wpb_waves, c->split, c->smem, &max_blocks));
    REGC_CHECK(max_blocks >= c->nblocks, REGC_EUNSUPPORTED,
               "a persistent launch needs all %d workgroups resident at once; the device holds %d", c->nblocks,
               max_blocks);
    REGC_CHECK(a.n_class <= c->nblocks, REGC_EUNSUPPORTED, "fewer workgroups than classes");
    int rc;
    // the barrier starts from zero arrivals (also after a launch that reported a
    // timed-out wait)
    REGC_HIP(hipMemsetAsync(c->gbar_d.p, 0, sizeof(unsigned int) * 2, c->stream));
    if (c->timing && (rc = record_event(c, c->ev_sweep, true))) return rc;
    if (c->balance) {
        REGC_HIP(launch_balance(c->cls_d.p, (int)c->cls.size(), c->n_d.p, c->wpb, c->wslot_d.p, c->stream));
        a.wslot = c->wslot_d.p;
    }
    if (c->opts.precision == REGC_FP64)
        REGC_HIP(launch_sweep_persist_f64(a, c->nblocks, wpb_waves, c->split, c->smem, c->stream));
    else
        REGC_HIP(launch_sweep_persist_f32(a, c->nblocks, wpb_waves, c->split, c->smem, c->stream));
    if (c->timing && (rc = record_event(c, c->ev_sweep, false))) return rc;
    c->persist_used = true;
    return REGC_OK;
}

// Philox4x32-10 on the host (the published definition: ten rounds of the two
// multiplications 0xD2511F53 and 0xCD9E8D57, Weyl key increments 0x9E3779B9 and
// 0xBB67AE85), for the paper schedule's per-step coin.
static void philox_host(uint32_t c[4], uint32_t k0, uint32_t k1)
{
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = (uint64_t)0xD2511F53u * c[0];
        const uint64_t pb = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n0 = (uint32_t)(pb >> 32) ^ c[1] ^ k0, n1 = (uint32_t)pb;
        const uint32_t n2 = (uint32_t)(pa >> 32) ^ c[3] ^ k1, n3 = (uint32_t)pa;
        c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// true when step q of the paper schedule is a particle-exchange (grand-canonical)
// step, false when it is a replica-exchange step
static bool paper_step_is_gc(const regc_ctx *c, int64_t q)
{
    uint32_t w[4] = {0u, (uint32_t)q, 0xFFFFFFFFu, 6u};
    philox_host(w, (uint32_t)c->opts.seed, (uint32_t)(c->opts.seed >> 32));
    return ((double)w[0] + 0.5) * (1.0 / 4294967296.0) < c->opts.x0;
}

// Observables of every walker for the record that ends at `sweep` (a sample point).
static int launch_obs_record(regc_ctx *c, int64_t sweep, hipStream_t stream)
{
    const regc_opts &o = c->opts;
    if (o.sample_every <= 0 || sweep % o.sample_every != 0 || sweep == 0) return REGC_OK;
    if (c->min_on) {
        MinArgs m{};
        m.walker_class = c->walker_class_d.p;
        m.n_walkers = c->W;
        m.n_class = (int)c->cls.size();
        m.nN = c->nmax_all + 1;
        m.n = c->n_d.p;
        m.e = c->e_d.p;
        m.xyz = c->xyz_d.p;
        m.xyz_stride = c->nmax_all;
        m.key = c->minkey_d.p;
        m.old_key = c->minold_d.p;
        m.widx = c->minw_d.p;
        m.e_min = c->mine_d.p;
        m.xyz_min = c->minxyz_d.p;
        REGC_HIP(launch_minima(m, stream));
    }
    if (!c->obs_on) return REGC_OK;
    const int64_t rec = sweep / o.sample_every - 1 - c->rec_base;
    REGC_CHECK(rec >= 0 && rec < c->rec_cap, REGC_ECAPACITY, "observable record %lld outside the buffer",
               (long long)rec);
    ObsArgs a{};
    a.cls = c->cls_d.p;
    a.walker_class = c->walker_class_d.p;
    a.n_walkers = c->W;
    a.n = c->n_d.p;
    a.xyz = c->xyz_d.p;
    a.xyz_stride = c->nmax_all;
    a.dz = c->obs_spec.dz;
    a.layer_lo = c->obs_spec.layer_lo;
    a.layer_hi = c->obs_spec.layer_hi;
    a.dr = c->obs_spec.dr;
    a.n_z = c->obs_nz;
    a.n_r = c->obs_spec.n_r;
    a.n_obs = c->n_obs;
    a.out = c->obs_d.p + (size_t)rec * c->W * c->n_obs;
    REGC_HIP(launch_observables(a, stream));
    return REGC_OK;
}

// The captured graph bakes in the sample and trace bases: drop it when they move.
static void invalidate_graph(regc_ctx *c)
{
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
}

// Captures graph_intervals exchange intervals (sweep launches, exchange, clock
// advance) once; replays start from the sweep index held in the device clock.
static int build_graph(regc_ctx *c)
{
    if (c->gexec) return REGC_OK;
    const regc_opts &o = c->opts;
    const int spl = o.sweeps_per_launch > 0 ? std::min(o.sweeps_per_launch, o.swap_every) : o.swap_every;
    REGC_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    REGC_HIP(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = REGC_OK;
    for (int r = 0; r < o.graph_intervals && !rc; ++r) {
        for (int off = 0; off < o.swap_every && !rc; off += spl)
            rc = launch_sweeps(c, off, std::min(spl, o.swap_every - off), c->cap_stream, true);
        if (!rc) rc = launch_exchange(c, 0, c->cap_stream, true);
        if (!rc && launch_clock_advance(c->clock_d.p, o.swap_every, c->cap_stream) != hipSuccess) rc = REGC_EHIP;
    }
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    REGC_CHECK(e == hipSuccess, REGC_EHIP, "graph capture failed: %s", hipGetErrorString(e));
    c->graph = g;
    REGC_HIP(hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
    return REGC_OK;
}

extern "C" int regc_run(regc_ctx *c, int64_t n_sweeps)
{
    REGC_CHECK(c, REGC_EINVAL, "null context");
    REGC_CHECK(n_sweeps >= 0, REGC_EINVAL, "negative sweep count");
    const regc_opts &o = c->opts;
    if (o.sample_every > 0) {
        const int64_t recs = (c->sweep + n_sweeps) / o.sample_every - c->sweep / o.sample_every;
        REGC_CHECK(c->n_rec + recs <= c->rec_cap, REGC_ECAPACITY,
                   "samples of %lld more records do not fit (%lld of %lld held)", (long long)recs,
                   (long long)c->n_rec, (long long)c->rec_cap);
    }
    if (c->trace_cap > 0)
        REGC_CHECK(c->sweep + n_sweeps - c->trace_sweep0 <= c->trace_cap, REGC_ECAPACITY,
                   "trace capacity of %lld sweeps exceeded", (long long)c->trace_cap);
    if (o.schedule == 1) {
        // runs of steps without an exchange step go to one launch; an exchange step
        // runs the exchange kernel first and starts the next launch
        const int spl = o.sweeps_per_launch > 0 ? o.sweeps_per_launch : 100;
        int64_t q = c->sweep;
        const int64_t end = c->sweep + n_sweeps;
        while (q < end) {
            int rc;
            if (!paper_step_is_gc(c, q) && (rc = launch_exchange(c, q, c->stream, false))) return rc;
            int64_t r = q + 1;
            while (r < end && r - q < spl && paper_step_is_gc(c, r) &&
                   !((c->obs_on || c->min_on) && o.sample_every > 0 && r % o.sample_every == 0))
                ++r;
            if ((rc = launch_sweeps(c, q, (int)(r - q), c->stream, false))) return rc;
            if ((rc = launch_obs_record(c, r, c->stream))) return rc;
            q = r;
        }
        c->sweep = end;
        if (o.sample_every > 0) c->n_rec = c->sweep / o.sample_every - c->rec_base;
        return REGC_OK;
    }
    int64_t left = n_sweeps;
    const bool persist = o.persistent > 0 && !learned_on(c) && !c->obs_on && !c->min_on;
    auto eager = [&](int64_t count) -> int {
        int64_t rem = count;
        while (rem > 0) {
            if (persist && c->sweep % o.swap_every == 0 && rem >= o.swap_every) {
                const int k = (int)std::min<int64_t>(o.persistent, rem / o.swap_every);
                const int rc = launch_persistent(c, c->sweep, k);
                if (rc) return rc;
                c->sweep += (int64_t)k * o.swap_every;
                rem -= (int64_t)k * o.swap_every;
                continue;
            }
            int64_t chunk = rem;
            if (o.swap_every > 0) chunk = std::min<int64_t>(chunk, o.swap_every - c->sweep % o.swap_every);
            const int spl = o.sweeps_per_launch > 0 ? o.sweeps_per_launch : (o.swap_every > 0 ? o.swap_every : 100);
            chunk = std::min<int64_t>(chunk, spl);
            if ((c->obs_on || c->min_on) && o.sample_every > 0)
                chunk = std::min<int64_t>(chunk, o.sample_every - c->sweep % o.sample_every);
            int rc = launch_sweeps(c, c->sweep, (int)chunk, c->stream, false);
            if (rc) return rc;
            c->sweep += chunk;
            if ((rc = launch_obs_record(c, c->sweep, c->stream))) return rc;
            rem -= chunk;
            if (o.swap_every > 0 && c->sweep % o.swap_every == 0) {
                rc = launch_exchange(c, c->sweep / o.swap_every - 1, c->stream, false);
                if (rc) return rc;
            }
        }
        return REGC_OK;
    };
    int rc;
    if (o.graph_intervals > 0 && o.swap_every > 0) {
        const int64_t align = (o.swap_every - c->sweep % o.swap_every) % o.swap_every;
        const int64_t pre = std::min(align, left);
        if ((rc = eager(pre))) return rc;
        left -= pre;
        const int64_t per = (int64_t)o.graph_intervals * o.swap_every;
        const int64_t reps = left / per;
        if (reps > 0) {
            if ((rc = build_graph(c))) return rc;
            REGC_HIP(launch_clock_set(c->clock_d.p, c->sweep, c->stream));
            for (int64_t r = 0; r < reps; ++r) {
                if (c->timing && (rc = record_event(c, c->ev_sweep, true))) return rc;
                REGC_HIP(hipGraphLaunch(c->gexec, c->stream));
                if (c->timing && (rc = record_event(c, c->ev_sweep, false))) return rc;
                c->sweep += per;
            }
            left -= reps * per;
        }
    }
    if ((rc = eager(left))) return rc;
    if (o.sample_every > 0) c->n_rec = c->sweep / o.sample_every - c->rec_base;
    return REGC_OK;
}

// Workgroup order of the learned kernel.  Workgroups are dispatched round-robin over
// the XCDs (workgroup b on XCD b mod n_xcd), each XCD with its own L2; a network pass
// streams the class's output layer (1 MB) from L2, and a batch's networks together
// exceed one XCD's L2.  So each class gets a set of XCDs in proportion to its walkers
// and its walkers go to workgroups on those XCDs: every XCD then streams (nearly) one
// network.  Single-class contexts keep the identity order.
static std::vector<int> xcd_walker_order(const std::vector<int> &walker_class, int n_class, int n_xcd)
{
    const int W = (int)walker_class.size();
    std::vector<int> order(W);
    for (int w = 0; w < W; ++w) order[w] = w;
    if (n_class <= 1 || n_xcd <= 1 || n_class > n_xcd) return order;
    std::vector<std::vector<int>> queue(n_class);
    for (int w = W - 1; w >= 0; --w) queue[walker_class[w]].push_back(w);     // popped from the back
    // XCDs per class: largest remainder, at least one each
    std::vector<int> share(n_class, 1);
    std::vector<double> rem(n_class);
    int left = n_xcd - n_class;
    for (int k = 0; k < n_class; ++k) {
        const double want = (double)queue[k].size() * n_xcd / W - 1.0;
        const int whole = want > 0 ? std::min((int)want, left) : 0;
        share[k] += whole;
        left -= whole;
        rem[k] = want - whole;
    }
    while (left > 0) {
        int best = 0;
        for (int k = 1; k < n_class; ++k)
            if (rem[k] > rem[best]) best = k;
        share[best] += 1;
        rem[best] -= 1.0;
        --left;
    }
    std::vector<int> xcd_class(n_xcd);
    for (int k = 0, x = 0; k < n_class; ++k)
        for (int j = 0; j < share[k]; ++j) xcd_class[x++] = k;
    for (int b = 0; b < W; ++b) {
        int k = xcd_class[b % n_xcd];
        if (queue[k].empty()) {                 // this class is done: the fullest other one
            for (int q = 0; q < n_class; ++q)
                if (queue[q].size() > queue[k].size()) k = q;
        }
        order[b] = queue[k].back();
        queue[k].pop_back();
    }
    return order;
}

// Installs (mlp, alpha) as the insertion proposal of class cls, or of every class
// when cls < 0; mlp = NULL or alpha = 0 removes it.
static int set_proposal(regc_ctx *c, int cls, regc_mlp *mlp, double alpha)
{
    REGC_CHECK(c, REGC_EINVAL, "null context");
    REGC_CHECK(alpha >= 0.0 && alpha <= 1.0, REGC_EINVAL, "mixture weight %g outside [0, 1]", alpha);
    REGC_CHECK(cls < (int)c->cls.size(), REGC_EINVAL, "class index %d out of range", cls);
    REGC_HIP(hipStreamSynchronize(c->stream));
    invalidate_graph(c);
    c->alpha.resize(c->cls.size(), 0.0);
    const int k0 = cls < 0 ? 0 : cls, k1 = cls < 0 ? (int)c->cls.size() : cls + 1;
    if (!mlp || alpha == 0.0) {
        for (int k = k0; k < k1; ++k) c->alpha[k] = 0.0;
        return REGC_OK;
    }
    REGC_CHECK(c->cls.size() <= (size_t)kMaxLearnClasses, REGC_EUNSUPPORTED,
               "the learned proposal takes at most %d classes", kMaxLearnClasses);
    REGC_CHECK(c->opts.schedule == 0, REGC_EUNSUPPORTED, "the learned proposal runs with the sweep schedule");
    int dev = 0, lds_max = 0;
    REGC_HIP(hipGetDevice(&dev));
    REGC_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const int real = c->opts.precision == REGC_FP64 ? 8 : 4;
    const size_t smem = learn_lds(c->max_slab_len, c->nmax_all, real).total;
    REGC_CHECK(smem <= (size_t)lds_max, REGC_EUNSUPPORTED, "a walker needs %zu bytes of LDS, the device allows %d",
               smem, lds_max);
    int rc;
    const size_t ncls = c->cls.size();
    if (!c->net_w.p && (rc = c->net_w.alloc(ncls * kNetWords))) return rc;
    if (!c->net_b.p && (rc = c->net_b.alloc(ncls * kNetBiases))) return rc;
    if (!c->net_ev_d.p) {
        if ((rc = c->net_ev_d.alloc(4))) return rc;
        REGC_HIP(hipMemset(c->net_ev_d.p, 0, 4 * sizeof(unsigned long long)));
    }
    if (!c->learn_order_d.p) {
        int n_cu = 0;
        REGC_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
        const int n_xcd = n_cu % 32 == 0 ? std::max(1, n_cu / 32) : 1;      // 32 CUs per XCD on CDNA4
        const std::vector<int> order = xcd_walker_order(c->walker_class, (int)ncls, n_xcd);
        if ((rc = c->learn_order_d.alloc(order.size())) ||
            (rc = upload(c->learn_order_d.p, order.data(), sizeof(int) * order.size())))
            return rc;
    }
    for (int k = k0; k < k1; ++k) {
        uint16_t *w = c->net_w.p + (size_t)k * kNetWords;
        float *b = c->net_b.p + (size_t)k * kNetBiases;
        if ((rc = mlp_export_sampler(mlp, c->opts.precision == REGC_FP64, w, w + (size_t)kNetNV * kNetH,
                                     w + (size_t)kNetNV * kNetH + kNetH * kNetH,
                                     w + (size_t)kNetNV * kNetH + 2 * kNetH * kNetH, b, b + kNetH, b + 2 * kNetH,
                                     b + 3 * kNetH, c->stream)))
            return rc;
        c->alpha[k] = alpha;
    }
    REGC_HIP(hipStreamSynchronize(c->stream));
    c->learn_smem = smem;
    return REGC_OK;
}

extern "C" int regc_set_proposal(regc_ctx *c, regc_mlp *mlp, double alpha)
{
    return set_proposal(c, -1, mlp, alpha);
}

extern "C" int regc_proposal_eval(regc_ctx *c, int cls, int n_conf, const int32_t *n, const double *xyz,
                                  const int32_t *skip, float *logits, double *lse, double *lnp)
{
    REGC_CHECK(c && n && xyz && skip && logits && lse && lnp, REGC_EINVAL, "null argument");
    REGC_CHECK(cls >= 0 && cls < (int)c->cls.size(), REGC_EINVAL, "class index %d out of range", cls);
    REGC_CHECK(cls < (int)c->alpha.size() && c->alpha[cls] > 0.0, REGC_ESTATE, "class %d has no network", cls);
    REGC_CHECK(n_conf > 0, REGC_EINVAL, "no configurations");
    const ClassHost &h = c->cls[cls];
    const int stride = c->nmax_all;
    for (int k = 0; k < n_conf; ++k) {
        REGC_CHECK(n[k] >= 0 && n[k] <= h.sys.n_max, REGC_EINVAL, "configuration %d: N out of range", k);
        REGC_CHECK(skip[k] >= -1 && skip[k] < std::max(n[k], 1), REGC_EINVAL, "configuration %d: bad skip", k);
    }
    DevBuf<double> x_d, lse_d, lnp_d;
    DevBuf<int32_t> n_d, s_d;
    DevBuf<float> lg_d;
    int rc;
    const size_t nv = (size_t)n_conf * kNetNV;
    if ((rc = x_d.alloc((size_t)n_conf * stride * 3)) || (rc = lse_d.alloc(n_conf)) || (rc = lnp_d.alloc(nv)) ||
        (rc = n_d.alloc(n_conf)) || (rc = s_d.alloc(n_conf)) || (rc = lg_d.alloc(nv)))
        return rc;
    REGC_HIP(hipMemcpy(x_d.p, xyz, sizeof(double) * (size_t)n_conf * stride * 3, hipMemcpyHostToDevice));
    REGC_HIP(hipMemcpy(n_d.p, n, sizeof(int32_t) * n_conf, hipMemcpyHostToDevice));
    REGC_HIP(hipMemcpy(s_d.p, skip, sizeof(int32_t) * n_conf, hipMemcpyHostToDevice));
    const uint16_t *w = c->net_w.p + (size_t)cls * kNetWords;
    const float *bb = c->net_b.p + (size_t)cls * kNetBiases;
    NetDev d;
    d.w1 = w;
    d.w2 = w + (size_t)kNetNV * kNetH;
    d.w3 = d.w2 + (size_t)kNetH * kNetH;
    d.w4 = d.w3 + (size_t)kNetH * kNetH;
    d.b1 = bb;
    d.b2 = bb + kNetH;
    d.b3 = bb + 2 * kNetH;
    d.b4 = bb + 3 * kNetH;
    REGC_HIP(hipStreamSynchronize(c->stream));
    if (c->opts.precision == REGC_FP64)
        REGC_HIP(launch_net_eval_f64(d, c->cls_d.p, cls, stride, n_conf, x_d.p, n_d.p, s_d.p, lg_d.p, lse_d.p,
                                     lnp_d.p, c->stream));
    else
        REGC_HIP(launch_net_eval_f32(d, c->cls_d.p, cls, stride, n_conf, x_d.p, n_d.p, s_d.p, lg_d.p, lse_d.p,
                                     lnp_d.p, c->stream));
    REGC_HIP(hipStreamSynchronize(c->stream));
    REGC_HIP(hipMemcpy(logits, lg_d.p, sizeof(float) * nv, hipMemcpyDeviceToHost));
    REGC_HIP(hipMemcpy(lse, lse_d.p, sizeof(double) * n_conf, hipMemcpyDeviceToHost));
    REGC_HIP(hipMemcpy(lnp, lnp_d.p, sizeof(double) * nv, hipMemcpyDeviceToHost));
    return REGC_OK;
}

extern "C" int regc_set_class_proposal(regc_ctx *c, int cls, regc_mlp *mlp, double alpha)
{
    REGC_CHECK(cls >= 0, REGC_EINVAL, "class index %d out of range", cls);
    return set_proposal(c, cls, mlp, alpha);
}

extern "C" int regc_set_observables(regc_ctx *c, const regc_observables *spec)
{
    REGC_CHECK(c, REGC_EINVAL, "null context");
    if (!spec) {
        c->obs_on = false;
        return REGC_OK;
    }
    REGC_CHECK(c->opts.graph_intervals == 0, REGC_EUNSUPPORTED, "observables are not recorded in graph replay");
    REGC_CHECK(c->opts.sample_every > 0 && c->rec_cap > 0, REGC_ESTATE, "the context records no samples");
    REGC_CHECK(spec->dz > 0 && spec->dr > 0 && spec->n_r >= 0 && spec->layer_hi >= spec->layer_lo, REGC_EINVAL,
               "bad observable spec");
    int nz = 0;
    for (auto &k : c->cls) nz = std::max(nz, (int)std::ceil((k.sys.z_hi - k.sys.z_lo) / spec->dz));
    const int n_obs = nz + spec->n_r + 1;
    REGC_CHECK(n_obs <= 2048, REGC_EINVAL, "%d observable bins (at most 2048)", n_obs);
    REGC_HIP(hipStreamSynchronize(c->stream));
    int rc;
    if (n_obs != c->n_obs || !c->obs_d.p) {
        if ((rc = c->obs_d.alloc((size_t)c->rec_cap * c->W * n_obs))) return rc;
    }
    REGC_HIP(hipMemset(c->obs_d.p, 0, sizeof(uint32_t) * (size_t)c->rec_cap * c->W * n_obs));
    c->obs_spec = *spec;
    c->obs_nz = nz;
    c->n_obs = n_obs;
    c->obs_on = true;
    return REGC_OK;
}

extern "C" int regc_observables_device(regc_ctx *c, const uint32_t **obs_dev, int *n_obs)
{
    REGC_CHECK(c && obs_dev && n_obs, REGC_EINVAL, "null argument");
    REGC_HIP(hipStreamSynchronize(c->stream));
    *obs_dev = c->obs_d.p;
    *n_obs = c->n_obs;
    return REGC_OK;
}

extern "C" int regc_track_minima(regc_ctx *c, int on)
{
    REGC_CHECK(c, REGC_EINVAL, "null context");
    if (!on) {
        c->min_on = false;
        return REGC_OK;
    }
    REGC_CHECK(c->opts.graph_intervals == 0, REGC_EUNSUPPORTED, "minima are not tracked in graph replay");
    REGC_CHECK(c->opts.sample_every > 0, REGC_ESTATE, "the context records no samples");
    REGC_HIP(hipStreamSynchronize(c->stream));
    if (!c->minkey_d.p) {
        const size_t slots = c->cls.size() * (size_t)(c->nmax_all + 1);
        int rc;
        if ((rc = c->minkey_d.alloc(slots)) || (rc = c->minold_d.alloc(slots)) || (rc = c->minw_d.alloc(slots)) ||
            (rc = c->mine_d.alloc(slots)) || (rc = c->minxyz_d.alloc(slots * c->nmax_all * 3)))
            return rc;
        std::vector<unsigned long long> k(slots, ~0ull);
        std::vector<int> wi(slots, 0x7fffffff);
        std::vector<double> e(slots, HUGE_VAL);
        REGC_HIP(hipMemcpy(c->minkey_d.p, k.data(), slots * sizeof(unsigned long long), hipMemcpyHostToDevice));
        REGC_HIP(hipMemcpy(c->minw_d.p, wi.data(), slots * sizeof(int), hipMemcpyHostToDevice));
        REGC_HIP(hipMemcpy(c->mine_d.p, e.data(), slots * sizeof(double), hipMemcpyHostToDevice));
        REGC_HIP(hipMemset(c->minxyz_d.p, 0, slots * c->nmax_all * 3 * sizeof(double)));
    }
    c->min_on = true;
    return REGC_OK;
}

extern "C" int regc_get_minima(regc_ctx *c, int cls, double *e_min, double *xyz)
{
    REGC_CHECK(c && e_min, REGC_EINVAL, "null argument");
    REGC_CHECK(cls >= 0 && cls < (int)c->cls.size(), REGC_EINVAL, "class index out of range");
    REGC_CHECK(c->minkey_d.p, REGC_ESTATE, "minima are not tracked");
    REGC_HIP(hipStreamSynchronize(c->stream));
    const size_t nN = c->nmax_all + 1, nmc = c->cls[cls].sys.n_max;
    std::vector<double> e(nN);
    REGC_HIP(hipMemcpy(e.data(), c->mine_d.p + cls * nN, nN * sizeof(double), hipMemcpyDeviceToHost));
    for (size_t N = 0; N <= nmc; ++N) e_min[N] = e[N];
    if (xyz) {
        std::vector<double> x(nN * c->nmax_all * 3);
        REGC_HIP(hipMemcpy(x.data(), c->minxyz_d.p + cls * nN * c->nmax_all * 3, x.size() * sizeof(double),
                           hipMemcpyDeviceToHost));
        for (size_t N = 0; N <= nmc; ++N)
            for (size_t j = 0; j < nmc * 3; ++j) xyz[(N * nmc) * 3 + j] = x[(N * c->nmax_all) * 3 + j];
    }
    return REGC_OK;
}

extern "C" int regc_aiat_phase(const double *e_min, int n_max, int n_mu, const double *mu, int32_t *phase)
{
    REGC_CHECK(e_min && mu && phase && n_max >= 0 && n_mu >= 0, REGC_EINVAL, "bad argument");
    const double e0 = e_min[0] < HUGE_VAL ? e_min[0] : 0.0;
    for (int m = 0; m < n_mu; ++m) {
        double best = HUGE_VAL;
        int arg = -1;
        for (int N = 0; N <= n_max; ++N) {
            if (!(e_min[N] < HUGE_VAL)) continue;
            const double g = e_min[N] - e0 - (double)N * mu[m];
            if (g < best) {
                best = g;
                arg = N;
            }
        }
        phase[m] = arg;
    }
    return REGC_OK;
}

extern "C" int regc_get_observables(regc_ctx *c, uint32_t *obs, int64_t cap_records, int64_t *n_out)
{
    REGC_CHECK(c && obs && n_out, REGC_EINVAL, "null argument");
    REGC_CHECK(c->obs_d.p && c->n_obs > 0, REGC_ESTATE, "no observables recorded");
    REGC_HIP(hipStreamSynchronize(c->stream));
    const int64_t k = std::min(cap_records, c->n_rec);
    REGC_HIP(hipMemcpy(obs, c->obs_d.p, sizeof(uint32_t) * (size_t)k * c->W * c->n_obs, hipMemcpyDeviceToHost));
    *n_out = k;
    return REGC_OK;
}

extern "C" int regc_capture_voxels(regc_ctx *c, uint16_t *vox_dev, int32_t *n_dev)
{
    REGC_CHECK(c && vox_dev && n_dev, REGC_EINVAL, "null argument");
    REGC_HIP(launch_capture_voxels(c->W, c->nmax_all, c->cls_d.p, c->walker_class_d.p, c->n_d.p, c->xyz_d.p,
                                   c->nmax_all, vox_dev, n_dev, c->stream));
    return REGC_OK;
}

extern "C" int regc_get_proposal_stats(regc_ctx *c, int64_t counts[4])
{
    REGC_CHECK(c && counts, REGC_EINVAL, "null argument");
    unsigned long long h[4] = {0, 0, 0, 0};
    REGC_HIP(hipStreamSynchronize(c->stream));
    if (c->net_ev_d.p) REGC_HIP(hipMemcpy(h, c->net_ev_d.p, sizeof h, hipMemcpyDeviceToHost));
    for (int k = 0; k < 4; ++k) counts[k] = (int64_t)h[k];
    return REGC_OK;
}

extern "C" int regc_sync(regc_ctx *c)
{
    REGC_CHECK(c, REGC_EINVAL, "null context");
    REGC_HIP(hipStreamSynchronize(c->stream));
    if (c->persist_used) {
        int err = 0;
        REGC_HIP(hipMemcpy(&err, c->gerr_d.p, sizeof(int), hipMemcpyDeviceToHost));
        REGC_CHECK(!err, REGC_EHIP, "a grid barrier of a persistent launch waited past its bound");
    }
    return REGC_OK;
}

extern "C" int regc_get_sweep(const regc_ctx *c, int64_t *sweep)
{
    REGC_CHECK(c && sweep, REGC_EINVAL, "null argument");
    *sweep = c->sweep;
    return REGC_OK;
}

extern "C" int regc_get_walkers(regc_ctx *c, int32_t *n, double *e, int32_t *label, double *xyz)
{
    REGC_CHECK(c, REGC_EINVAL, "null context");
    REGC_HIP(hipStreamSynchronize(c->stream));
    if (n) REGC_HIP(hipMemcpy(n, c->n_d.p, sizeof(int32_t) * c->W, hipMemcpyDeviceToHost));
    if (e) REGC_HIP(hipMemcpy(e, c->e_d.p, sizeof(double) * c->W, hipMemcpyDeviceToHost));
    if (label) REGC_HIP(hipMemcpy(label, c->label_d.p, sizeof(int32_t) * c->W, hipMemcpyDeviceToHost));
    if (xyz) {
        REGC_HIP(hipMemcpy(xyz, c->xyz_d.p, sizeof(double) * (size_t)c->W * c->nmax_all * 3, hipMemcpyDeviceToHost));
        std::vector<int32_t> nn(c->W);
        REGC_HIP(hipMemcpy(nn.data(), c->n_d.p, sizeof(int32_t) * c->W, hipMemcpyDeviceToHost));
        for (int w = 0; w < c->W; ++w)
            std::fill(xyz + ((size_t)w * c->nmax_all + nn[w]) * 3, xyz + ((size_t)w + 1) * c->nmax_all * 3, 0.0);
    }
    return REGC_OK;
}

static int run_energy(regc_ctx *c, double *e_dev)
{
    EnergyArgs a{};
    a.cls = c->cls_d.p;
    a.walker_class = c->walker_class_d.p;
    a.n_walkers = c->W;
    a.pot = c->potd;
    a.n = c->n_d.p;
    a.xyz = c->xyz_d.p;
    a.xyz_stride = c->nmax_all;
    a.slab4 = c->unb_d.p;
    a.unb_off = c->unb_off_d.p;
    a.unb_len = c->unb_len_d.p;
    a.e_out = e_dev;
    if (c->opts.precision == REGC_FP64)
        REGC_HIP(launch_energy_f64(a, c->stream));
    else
        REGC_HIP(launch_energy_f32(a, c->stream));
    return REGC_OK;
}

extern "C" int regc_set_walkers(regc_ctx *c, const int32_t *n, const double *xyz, const int32_t *label)
{
    REGC_CHECK(c && n && xyz, REGC_EINVAL, "null argument");
    for (int w = 0; w < c->W; ++w) {
        const ClassHost &h = c->cls[c->walker_class[w]];
        REGC_CHECK(n[w] >= 0 && n[w] <= h.sys.n_max, REGC_EINVAL, "walker %d: N out of range", w);
        for (int k = 0; k < n[w]; ++k) {
            const double *p = xyz + ((size_t)w * c->nmax_all + k) * 3;
            REGC_CHECK(p[0] >= 0 && p[0] <= h.sys.lx && p[1] >= 0 && p[1] <= h.sys.ly && p[2] >= h.sys.z_lo &&
                           p[2] <= h.sys.z_hi,
                       REGC_EINVAL, "walker %d particle %d outside the gas region", w, k);
        }
    }
    std::vector<int32_t> wos;
    if (label) {
        wos.assign(c->W, -1);
        for (auto &h : c->cls)
            for (int w = 0; w < h.S; ++w) {
                const int s = label[h.off + w];
                REGC_CHECK(s >= 0 && s < h.S && wos[h.off + s] < 0, REGC_EINVAL, "labels are not a permutation");
                wos[h.off + s] = h.off + w;
            }
    }
    REGC_HIP(hipStreamSynchronize(c->stream));
    REGC_HIP(hipMemcpy(c->n_d.p, n, sizeof(int32_t) * c->W, hipMemcpyHostToDevice));
    REGC_HIP(hipMemcpy(c->xyz_d.p, xyz, sizeof(double) * (size_t)c->W * c->nmax_all * 3, hipMemcpyHostToDevice));
    if (label) {
        REGC_HIP(hipMemcpy(c->label_d.p, label, sizeof(int32_t) * c->W, hipMemcpyHostToDevice));
        REGC_HIP(hipMemcpy(c->wos_d.p, wos.data(), sizeof(int32_t) * c->W, hipMemcpyHostToDevice));
    }
    int rc = run_energy(c, c->e_d.p);
    if (rc) return rc;
    if (c->tv_d.p) REGC_HIP(hipMemsetAsync(c->tv_d.p, 0, sizeof(double) * c->W, c->stream));   // fresh velocities
    REGC_HIP(hipStreamSynchronize(c->stream));
    return REGC_OK;
}

extern "C" int regc_energies(regc_ctx *c, double *e_out)
{
    REGC_CHECK(c && e_out, REGC_EINVAL, "null argument");
    DevBuf<double> tmp;
    int rc;
    if ((rc = tmp.alloc(c->W))) return rc;
    if ((rc = run_energy(c, tmp.p))) return rc;
    REGC_HIP(hipStreamSynchronize(c->stream));
    REGC_HIP(hipMemcpy(e_out, tmp.p, sizeof(double) * c->W, hipMemcpyDeviceToHost));
    return REGC_OK;
}

extern "C" int regc_sample_count(const regc_ctx *c, int64_t *count)
{
    REGC_CHECK(c && count, REGC_EINVAL, "null argument");
    *count = c->n_rec * c->W;
    return REGC_OK;
}

extern "C" int regc_get_samples(regc_ctx *c, double *e, int32_t *n, int32_t *state, int64_t cap, int64_t *n_out)
{
    REGC_CHECK(c && n_out, REGC_EINVAL, "null argument");
    const int64_t cnt = std::min<int64_t>(cap, c->n_rec * c->W);
    REGC_HIP(hipStreamSynchronize(c->stream));
    if (cnt > 0) {
        if (e) REGC_HIP(hipMemcpy(e, c->samp_e.p, sizeof(double) * cnt, hipMemcpyDeviceToHost));
        if (n) REGC_HIP(hipMemcpy(n, c->samp_n.p, sizeof(int32_t) * cnt, hipMemcpyDeviceToHost));
        if (state) REGC_HIP(hipMemcpy(state, c->samp_s.p, sizeof(int32_t) * cnt, hipMemcpyDeviceToHost));
    }
    *n_out = cnt;
    return REGC_OK;
}

extern "C" int regc_samples_device(regc_ctx *c, const double **e_dev, const int32_t **n_dev,
                                   const int32_t **state_dev, int64_t *count)
{
    REGC_CHECK(c, REGC_EINVAL, "null context");
    if (e_dev) *e_dev = c->samp_e.p;
    if (n_dev) *n_dev = c->samp_n.p;
    if (state_dev) *state_dev = c->samp_s.p;
    if (count) *count = c->n_rec * c->W;
    return REGC_OK;
}

extern "C" int regc_clear_samples(regc_ctx *c)
{
    REGC_CHECK(c, REGC_EINVAL, "null context");
    REGC_HIP(hipStreamSynchronize(c->stream));
    c->rec_base = c->opts.sample_every > 0 ? c->sweep / c->opts.sample_every : 0;
    c->n_rec = 0;
    REGC_HIP(hipMemset(c->hist_d.p, 0, sizeof(unsigned long long) * (size_t)c->W * (c->nmax_all + 1)));
    c->trace_sweep0 = c->sweep;
    invalidate_graph(c);
    return REGC_OK;
}

extern "C" int regc_get_stats(regc_ctx *c, int64_t *stats, int64_t *swap_att, int64_t *swap_acc)
{
    REGC_CHECK(c, REGC_EINVAL, "null context");
    REGC_HIP(hipStreamSynchronize(c->stream));
    if (stats) REGC_HIP(hipMemcpy(stats, c->stats_d.p, sizeof(int64_t) * (size_t)c->W * kNStat, hipMemcpyDeviceToHost));
    if (swap_att) REGC_HIP(hipMemcpy(swap_att, c->att_d.p, sizeof(int64_t) * 4 * c->W, hipMemcpyDeviceToHost));
    if (swap_acc) REGC_HIP(hipMemcpy(swap_acc, c->acc_d.p, sizeof(int64_t) * 4 * c->W, hipMemcpyDeviceToHost));
    return REGC_OK;
}

extern "C" int regc_count_pairs(regc_ctx *c, int on)
{
    REGC_CHECK(c, REGC_EINVAL, "null context");
    REGC_HIP(hipStreamSynchronize(c->stream));
    c->count_pairs = on != 0;
    invalidate_graph(c);
    return REGC_OK;
}

extern "C" int regc_get_pair_counts(regc_ctx *c, int64_t *candidates, int64_t *within_cutoff)
{
    REGC_CHECK(c, REGC_EINVAL, "null context");
    unsigned long long h[2];
    REGC_HIP(hipStreamSynchronize(c->stream));
    REGC_HIP(hipMemcpy(h, c->pairs_d.p, sizeof h, hipMemcpyDeviceToHost));
    if (candidates) *candidates = (int64_t)h[0];
    if (within_cutoff) *within_cutoff = (int64_t)h[1];
    return REGC_OK;
}

extern "C" int regc_get_histograms(regc_ctx *c, int64_t *n_hist)
{
    REGC_CHECK(c && n_hist, REGC_EINVAL, "null argument");
    REGC_HIP(hipStreamSynchronize(c->stream));
    REGC_HIP(hipMemcpy(n_hist, c->hist_d.p, sizeof(int64_t) * (size_t)c->W * (c->nmax_all + 1), hipMemcpyDeviceToHost));
    return REGC_OK;
}

extern "C" int regc_get_trace(regc_ctx *c, uint32_t *bits, int32_t *n_per_sweep, int64_t cap_sweeps, int64_t *n_out)
{
    REGC_CHECK(c && n_out, REGC_EINVAL, "null argument");
    REGC_CHECK(c->trace_cap > 0, REGC_ESTATE, "context created without a trace buffer");
    const int64_t have = std::min<int64_t>(c->sweep - c->trace_sweep0, c->trace_cap);
    const int64_t cnt = std::min<int64_t>(have, cap_sweeps);
    REGC_HIP(hipStreamSynchronize(c->stream));
    if (cnt > 0) {
        if (bits)
            REGC_HIP(hipMemcpy(bits, c->trace_bits_d.p, sizeof(uint32_t) * (size_t)cnt * c->W * c->words,
                               hipMemcpyDeviceToHost));
        if (n_per_sweep)
            REGC_HIP(hipMemcpy(n_per_sweep, c->trace_n_d.p, sizeof(int32_t) * (size_t)cnt * c->W, hipMemcpyDeviceToHost));
    }
    *n_out = cnt;
    return REGC_OK;
}

extern "C" int regc_timing_enable(regc_ctx *c, int enable)
{
    REGC_CHECK(c, REGC_EINVAL, "null context");
    REGC_HIP(hipStreamSynchronize(c->stream));
    for (auto &p : c->ev_sweep) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
    for (auto &p : c->ev_swap) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
    c->ev_sweep.clear();
    c->ev_swap.clear();
    c->timing = enable != 0;
    return REGC_OK;
}

extern "C" int regc_timing_get(regc_ctx *c, double *ms_sweep, int64_t *n_sweep, double *ms_swap, int64_t *n_swap)
{
    REGC_CHECK(c, REGC_EINVAL, "null context");
    REGC_HIP(hipStreamSynchronize(c->stream));
    double a = 0, b = 0;
    for (auto &p : c->ev_sweep) {
        float ms = 0;
        REGC_HIP(hipEventElapsedTime(&ms, p.a, p.b));
        a += ms;
    }
    for (auto &p : c->ev_swap) {
        float ms = 0;
        REGC_HIP(hipEventElapsedTime(&ms, p.a, p.b));
        b += ms;
    }
    if (ms_sweep) *ms_sweep = a;
    if (n_sweep) *n_sweep = (int64_t)c->ev_sweep.size();
    if (ms_swap) *ms_swap = b;
    if (n_swap) *n_swap = (int64_t)c->ev_swap.size();
    return REGC_OK;
}

// checkpoint layout: header, then n, e, label, wos, xyz, stats, att, acc
namespace {
struct CkptHeader {
    uint64_t magic;
    uint32_t version, W, nmax, n_class;
    int64_t sweep;
    uint64_t seed;
};
constexpr uint64_t kMagic = 0x3143474552ULL;   // "REGC1"
}  // namespace

static size_t ckpt_size(const regc_ctx *c)
{
    const size_t W = c->W;
    return sizeof(CkptHeader) + W * (4 + 8 + 4 + 4) + W * c->nmax_all * 3 * 8 + W * kNStat * 8 + 2 * 4 * W * 8;
}

extern "C" int regc_checkpoint(regc_ctx *c, void *buf, size_t cap, size_t *size)
{
    REGC_CHECK(c && size, REGC_EINVAL, "null argument");
    *size = ckpt_size(c);
    if (!buf) return REGC_OK;
    REGC_CHECK(cap >= *size, REGC_ECAPACITY, "checkpoint needs %zu bytes", *size);
    REGC_HIP(hipStreamSynchronize(c->stream));
    char *p = (char *)buf;
    CkptHeader h{kMagic, 1u, (uint32_t)c->W, (uint32_t)c->nmax_all, (uint32_t)c->cls.size(), c->sweep, c->opts.seed};
    std::memcpy(p, &h, sizeof h);
    p += sizeof h;
    const size_t W = c->W;
    REGC_HIP(hipMemcpy(p, c->n_d.p, W * 4, hipMemcpyDeviceToHost)); p += W * 4;
    REGC_HIP(hipMemcpy(p, c->e_d.p, W * 8, hipMemcpyDeviceToHost)); p += W * 8;
    REGC_HIP(hipMemcpy(p, c->label_d.p, W * 4, hipMemcpyDeviceToHost)); p += W * 4;
    REGC_HIP(hipMemcpy(p, c->wos_d.p, W * 4, hipMemcpyDeviceToHost)); p += W * 4;
    REGC_HIP(hipMemcpy(p, c->xyz_d.p, W * c->nmax_all * 3 * 8, hipMemcpyDeviceToHost)); p += W * c->nmax_all * 3 * 8;
    REGC_HIP(hipMemcpy(p, c->stats_d.p, W * kNStat * 8, hipMemcpyDeviceToHost)); p += W * kNStat * 8;
    REGC_HIP(hipMemcpy(p, c->att_d.p, 4 * W * 8, hipMemcpyDeviceToHost)); p += 4 * W * 8;
    REGC_HIP(hipMemcpy(p, c->acc_d.p, 4 * W * 8, hipMemcpyDeviceToHost));
    return REGC_OK;
}

extern "C" int regc_restore(regc_ctx *c, const void *buf, size_t size)
{
    REGC_CHECK(c && buf, REGC_EINVAL, "null argument");
    REGC_CHECK(size == ckpt_size(c), REGC_EINVAL, "checkpoint size does not match this context");
    const char *p = (const char *)buf;
    CkptHeader h;
    std::memcpy(&h, p, sizeof h);
    p += sizeof h;
    REGC_CHECK(h.magic == kMagic && h.version == 1 && h.W == (uint32_t)c->W && h.nmax == (uint32_t)c->nmax_all &&
                   h.n_class == (uint32_t)c->cls.size() && h.seed == c->opts.seed,
               REGC_EINVAL, "checkpoint was written by a different context");
    const size_t W = c->W;
    {
        // the kernels index LDS by N and the state arrays by label: check both, and
        // that walker-of-state inverts the labels, before anything reaches the device
        std::vector<int32_t> nn(W), lab(W), wos(W);
        std::memcpy(nn.data(), p, W * 4);
        std::memcpy(lab.data(), p + W * 12, W * 4);
        std::memcpy(wos.data(), p + W * 16, W * 4);
        REGC_CHECK(h.sweep >= 0, REGC_EINVAL, "checkpoint holds a negative sweep count");
        for (const ClassHost &k : c->cls)
            for (int w = k.off; w < k.off + k.S; ++w) {
                REGC_CHECK(nn[w] >= 0 && nn[w] <= k.sys.n_max, REGC_EINVAL, "checkpoint: N = %d of walker %d outside 0..%d",
                           nn[w], w, k.sys.n_max);
                REGC_CHECK(lab[w] >= 0 && lab[w] < k.S && wos[k.off + lab[w]] == w, REGC_EINVAL,
                           "checkpoint: label %d of walker %d is not a state of its class held by it", lab[w], w);
            }
    }
    REGC_HIP(hipStreamSynchronize(c->stream));
    REGC_HIP(hipMemcpy(c->n_d.p, p, W * 4, hipMemcpyHostToDevice)); p += W * 4;
    REGC_HIP(hipMemcpy(c->e_d.p, p, W * 8, hipMemcpyHostToDevice)); p += W * 8;
    REGC_HIP(hipMemcpy(c->label_d.p, p, W * 4, hipMemcpyHostToDevice)); p += W * 4;
    REGC_HIP(hipMemcpy(c->wos_d.p, p, W * 4, hipMemcpyHostToDevice)); p += W * 4;
    REGC_HIP(hipMemcpy(c->xyz_d.p, p, W * c->nmax_all * 3 * 8, hipMemcpyHostToDevice)); p += W * c->nmax_all * 3 * 8;
    REGC_HIP(hipMemcpy(c->stats_d.p, p, W * kNStat * 8, hipMemcpyHostToDevice)); p += W * kNStat * 8;
    REGC_HIP(hipMemcpy(c->att_d.p, p, 4 * W * 8, hipMemcpyHostToDevice)); p += 4 * W * 8;
    REGC_HIP(hipMemcpy(c->acc_d.p, p, 4 * W * 8, hipMemcpyHostToDevice));
    c->sweep = h.sweep;
    c->rec_base = c->opts.sample_every > 0 ? c->sweep / c->opts.sample_every : 0;
    c->n_rec = 0;
    c->trace_sweep0 = c->sweep;
    invalidate_graph(c);
    REGC_HIP(hipMemset(c->hist_d.p, 0, sizeof(unsigned long long) * W * (c->nmax_all + 1)));
    if (c->tv_d.p) REGC_HIP(hipMemset(c->tv_d.p, 0, sizeof(double) * W));   // velocities are not checkpointed
    return REGC_OK;
}

extern "C" void regc_destroy(regc_ctx *c)
{
    if (c) {
        (void)hipStreamSynchronize(c->stream);
        delete c;
    }
}

extern "C" int regc_mbar_load_run(regc_mbar *mb, regc_ctx *c, int cls, int64_t skip_records)
{
    REGC_CHECK(mb && c, REGC_EINVAL, "null argument");
    REGC_CHECK(cls >= 0 && cls < (int)c->cls.size(), REGC_EINVAL, "class index out of range");
    REGC_CHECK(skip_records >= 0 && skip_records < c->n_rec, REGC_EINVAL, "no records after the skipped ones");
    const int64_t recs = c->n_rec - skip_records;
    const int off = c->cls[cls].off, cnt = c->cls[cls].S;
    const size_t W = c->W;
    DevBuf<double> e;
    DevBuf<int32_t> n, s;
    int rc;
    if ((rc = e.alloc(recs * cnt)) || (rc = n.alloc(recs * cnt)) || (rc = s.alloc(recs * cnt))) return rc;
    REGC_HIP(hipStreamSynchronize(c->stream));
    REGC_HIP(hipMemcpy2D(e.p, cnt * sizeof(double), c->samp_e.p + skip_records * W + off, W * sizeof(double),
                         cnt * sizeof(double), recs, hipMemcpyDeviceToDevice));
    REGC_HIP(hipMemcpy2D(n.p, cnt * sizeof(int32_t), c->samp_n.p + skip_records * W + off, W * sizeof(int32_t),
                         cnt * sizeof(int32_t), recs, hipMemcpyDeviceToDevice));
    REGC_HIP(hipMemcpy2D(s.p, cnt * sizeof(int32_t), c->samp_s.p + skip_records * W + off, W * sizeof(int32_t),
                         cnt * sizeof(int32_t), recs, hipMemcpyDeviceToDevice));
    if ((rc = regc_mbar_set_samples(mb, recs * cnt, e.p, n.p, s.p, 1))) return rc;
    if (c->obs_d.p && c->n_obs > 0) {
        DevBuf<uint32_t> ob;
        const size_t no = c->n_obs;
        if ((rc = ob.alloc(recs * cnt * no))) return rc;
        REGC_HIP(hipMemcpy2D(ob.p, cnt * no * sizeof(uint32_t), c->obs_d.p + (skip_records * W + off) * no,
                             W * no * sizeof(uint32_t), cnt * no * sizeof(uint32_t), recs, hipMemcpyDeviceToDevice));
        if ((rc = regc_mbar_set_observables(mb, ob.p, (int)no, 1))) return rc;
    }
    return REGC_OK;
}
