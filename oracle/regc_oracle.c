/*
 * regc_oracle.c -- plain FP64 CPU oracle of the replica-exchange grand-canonical
 * (REGC) Monte Carlo method of Zhou, Scheffler and Ghiringhelli,
 * "Determining Surface Phase Diagrams Including Anharmonic Effects" (arXiv:1908.11118).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct reference
 * that the HIP library is checked against.  Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or constant generator with the HIP path.
 *
 * Everything is double precision, compiled without FP contraction and without
 * fast-math.  Each walker's chain is a plain sequential loop; OpenMP only runs
 * different walkers side by side between two sweep boundaries (walkers never
 * read each other's state there).
 *
 * What each function follows in the paper:
 *   - target distribution: Sec. II.A.1, Eq. (1) (GC probability density);
 *   - removal acceptance: Sec. II.A.1, Eq. (2); insertion acceptance: Eq. (3),
 *     read with the exponent beta*[mu - (E_{N+1} - E_N)] (the printed signs are
 *     garbled; this is the detailed-balance ratio of Eq. (1));
 *   - particle choice for removal: i = floor(y*N), Sec. II.A.1;
 *   - replica-exchange acceptance: Sec. II.A.2, Eq. (6), read as
 *     ln A = (b_a - b_b)(E_i - E_j) + (N_j - N_i)(lnz_a - lnz_b) with
 *     lnz = b*mu - 3 ln Lambda(T), Lambda = Lambda1/sqrt(T) (Eq. (1) again);
 *   - four collective neighbour-swap types chosen with probability 1/4,
 *     Sec. II.A.2 (Fig. 2 is not available; the types are read as even/odd
 *     T-axis pairs and even/odd mu-axis pairs);
 *   - displacement acceptance: Sec. II.A.3, Eq. (7), cube of half-width delta;
 *   - LJ 12-6 pair potential: Appendix, truncated and shifted at rc.
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), written
 * here from its published definition.
 *
 * Extension, not in the paper: a learned insertion proposal.  A network maps the
 * 16^3 occupancy grid of a configuration to a categorical over the 4096 voxels of
 * the gas region; an insertion point is either a voxel drawn from it plus a
 * uniform offset (probability alpha) or a uniform point of V, so its density is
 * q(r|X) = alpha P(v(r)|occ(X)) / V_vox + (1 - alpha) / V, and the acceptance
 * ratios of Eqs. (2)-(3) take the Metropolis-Hastings form
 *   insertion  ln A = ln z - ln(N+1) - ln q(r|X) - beta dE,
 *   removal    ln A = ln N + ln q(r_i|X without i) - ln z - beta dE,
 * which keeps Eq. (1) the stationary distribution for any network.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_NSTAT 10
enum {
    ST_DISP_ATT = 0, ST_DISP_ACC, ST_INS_ATT, ST_INS_ACC, ST_DEL_ATT, ST_DEL_ACC,
    ST_CAP_REJ, ST_EMPTY_REJ, ST_WALL_REJ, ST_CORE_REJ
};

/* ------------------------------------------------------------------------- */
/* Philox4x32-10                                                             */
/* ------------------------------------------------------------------------- */
/* One round maps (c0,c1,c2,c3) with key (k0,k1) to
 *   (hi(B*c2) ^ c1 ^ k0, lo(B*c2), hi(A*c0) ^ c3 ^ k1, lo(A*c0))
 * with A = 0xD2511F53, B = 0xCD9E8D57; between rounds the key is advanced by
 * the Weyl increments 0x9E3779B9 and 0xBB67AE85. Ten rounds. */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t pa = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t pb = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)pb;
        uint32_t n2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)pa;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void philox_words(uint64_t seed, uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t out[4])
{
    uint32_t ctr[4] = {a, b, c, d};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* open-interval uniform from one 32-bit word: (w + 1/2) / 2^32 (exact in FP64) */
static double u32_open(uint32_t w) { return ((double)w + 0.5) * (1.0 / 4294967296.0); }

/* 53-bit uniform in [0,1) from two words (exact in FP64) */
static double u53(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

/* ------------------------------------------------------------------------- */
/* Configuration                                                             */
/* ------------------------------------------------------------------------- */
typedef struct {
    /* pair potential (Appendix): phi(r) = 4 eps [(sig/r)^12 - (sig/r)^6] - shift, r < rc */
    double eps_gg, sig_gg, eps_gs, sig_gs, rc;
    int shifted;          /* 1: subtract phi(rc) so phi is continuous at rc */
    int mode;             /* 0 LJ gas on frozen LJ slab, 1 ideal gas (no interactions), 2 site lattice */
    double hc_frac;       /* new pairs closer than hc_frac*sigma are rejected outright */
    /* surface and gas region */
    int n_slab;
    const double *slab;   /* [n_slab][3] */
    double lx, ly, zlo, zhi;
    int n_sites;          /* mode 2 only */
    const double *sites;  /* [n_sites][3] */
    double lambda1;       /* thermal wavelength at T = 1 */
    int n_max;
    /* state grid: state s = l*n_mu + m */
    int n_t, n_mu;
    const double *t, *mu;
    /* schedule */
    uint64_t seed;
    double p_disp, p_ins, max_disp;
    int trials_per_sweep;
    int swap_every, sample_every, swap_scheme;
    /* position of this simulation inside a batch of several: its walkers' Philox
     * walker index is offset by walker_offset, its exchange stream is
     * 0xFFFFFFFF - class_id (both 0 for a lone simulation) */
    int walker_offset, class_id;
    /* learned insertion proposal: network parameters (FP32, layout below) or NULL,
     * and the mixture weight alpha of the network branch (0: plain method) */
    const float *net;
    double alpha;
    /* schedule: 0 = fixed-length sweeps of mixed trials (above); 1 = the paper's
     * REGC step: a global coin chooses, with probability x0, one particle-exchange
     * attempt per walker (removal or insertion with probability 1/2 each), else a
     * replica-exchange step; then mc_cycles cycles of N displacement attempts */
    int schedule;
    double x0;
    int mc_cycles;
    /* per-sample structural observables (Sec. III.A: axial density, lateral radial
     * distribution of a layer), recorded with every sample when obs_dz > 0:
     *   counts of particles in z bins of width obs_dz from zlo (n_z = ceil(H/dz)
     *   bins, the last one closed at zhi);
     *   counts of unordered pairs of particles both in the layer
     *   obs_layer_lo <= z < obs_layer_hi whose lateral minimum-image distance lies
     *   in [k dr, (k+1) dr), k < obs_nr;
     *   the number of particles in the layer. */
    double obs_dz, obs_layer_lo, obs_layer_hi, obs_dr;
    int obs_nr;
    /* canonical part of the paper's REGC step by molecular dynamics (Sec. II.A:
     * "S parallel molecular dynamics ... runs", Sec. II.A.3): md_steps > 0 replaces
     * the MC cycles by md_steps velocity-Verlet steps of md_dt (unit mass) with the
     * stochastic velocity-rescaling thermostat of time constant md_tau (0: none) */
    int md_steps;
    double md_dt, md_tau;
} orc_config;

/* derived per-state constants */
typedef struct {
    double beta, lnz;
} orc_statec;

static void state_constants(const orc_config *c, orc_statec *sc)
{
    for (int l = 0; l < c->n_t; ++l) {
        for (int m = 0; m < c->n_mu; ++m) {
            double T = c->t[l];
            double beta = 1.0 / T;
            double lnz;
            if (c->mode == 2) {
                lnz = beta * c->mu[m];                 /* site lattice: Lambda taken as 1 */
            } else {
                double lam = c->lambda1 / sqrt(T);     /* Lambda(T) = Lambda1 / sqrt(T) */
                lnz = beta * c->mu[m] - 3.0 * log(lam);
            }
            sc[l * c->n_mu + m].beta = beta;
            sc[l * c->n_mu + m].lnz = lnz;
        }
    }
}

double orc_state_lnz(double T, double mu, double lambda1, int mode)
{
    double beta = 1.0 / T;
    if (mode == 2) return beta * mu;
    return beta * mu - 3.0 * log(lambda1 / sqrt(T));
}

/* truncated (and optionally shifted) LJ 12-6 */
double orc_lj(double r2, double eps, double sig, double rc, int shifted)
{
    if (r2 >= rc * rc) return 0.0;
    double s2 = (sig * sig) / r2;
    double s6 = s2 * s2 * s2;
    double v = 4.0 * eps * (s6 * s6 - s6);
    if (shifted) {
        double c2 = (sig * sig) / (rc * rc);
        double c6 = c2 * c2 * c2;
        v -= 4.0 * eps * (c6 * c6 - c6);
    }
    return v;
}

static double min_image(double d, double box)
{
    if (d > 0.5 * box) return d - box;
    if (d < -0.5 * box) return d + box;
    return d;
}

static double dist2(const orc_config *c, const double *a, const double *b)
{
    double dx = min_image(a[0] - b[0], c->lx);
    double dy = min_image(a[1] - b[1], c->ly);
    double dz = a[2] - b[2];
    return dx * dx + dy * dy + dz * dz;
}

/* Interaction energy of a particle at p with the other gas particles (skip index `skip`)
 * and with the slab.  *core is set when a pair closer than the hard-core radius is found. */
static double particle_energy(const orc_config *c, const double *p, const double *xyz, int n,
                              int skip, int *core)
{
    double e = 0.0;
    double hg = c->hc_frac * c->sig_gg, hs = c->hc_frac * c->sig_gs;
    *core = 0;
    for (int j = 0; j < n; ++j) {
        if (j == skip) continue;
        double r2 = dist2(c, p, xyz + 3 * j);
        if (r2 < hg * hg) *core = 1;
        e += orc_lj(r2, c->eps_gg, c->sig_gg, c->rc, c->shifted);
    }
    for (int a = 0; a < c->n_slab; ++a) {
        double r2 = dist2(c, p, c->slab + 3 * a);
        if (r2 < hs * hs) *core = 1;
        e += orc_lj(r2, c->eps_gs, c->sig_gs, c->rc, c->shifted);
    }
    return e;
}

/* Total configurational energy: gas-gas pairs plus gas-slab pairs; the frozen
 * slab has no internal interaction (Sec. III.A). */
double orc_total_energy(const orc_config *c, int n, const double *xyz)
{
    if (c->mode == 1) return 0.0;
    double e = 0.0;
    for (int i = 0; i < n; ++i) {
        for (int j = i + 1; j < n; ++j)
            e += orc_lj(dist2(c, xyz + 3 * i, xyz + 3 * j), c->eps_gg, c->sig_gg, c->rc, c->shifted);
        for (int a = 0; a < c->n_slab; ++a)
            e += orc_lj(dist2(c, xyz + 3 * i, c->slab + 3 * a), c->eps_gs, c->sig_gs, c->rc, c->shifted);
    }
    return e;
}

/* ------------------------------------------------------------------------- */
/* Learned insertion proposal network                                        */
/* ------------------------------------------------------------------------- */
/* Parameter vector (FP32): W1 [4096][128] (row v: the weights of input voxel v),
 * b1 [128], W2 [128][128] ([out][in]), b2 [128], W3 [128][128], b3 [128],
 * W4 [4096][128] (row v: output voxel v), b4 [4096].
 * Arithmetic of the sampler's network: weights and hidden activations rounded
 * to bfloat16 (nearest, ties to even), products and sums in FP32, GELU in its
 * erf form; the log-normaliser and everything after it in FP64. */
#define NET_G 16
#define NET_NV (NET_G * NET_G * NET_G)
#define NET_H 128
#define NET_NPARAM ((size_t)NET_NV * NET_H + NET_H + 2 * ((size_t)NET_H * NET_H + NET_H) + (size_t)NET_NV * NET_H + NET_NV)

typedef struct {
    float *W1, *W2, *W3, *W4;        /* bfloat16-rounded copies */
    const float *b1, *b2, *b3, *b4;
} orc_net;

static float bf16_round(float x)
{
    uint32_t u;
    memcpy(&u, &x, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return x;          /* NaN */
    u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
    memcpy(&x, &u, 4);
    return x;
}

static float gelu(float x) { return 0.5f * x * (1.0f + (float)erf((double)x / sqrt(2.0))); }

static void net_prepare(const float *P, orc_net *net)
{
    const float *W1 = P, *b1 = W1 + (size_t)NET_NV * NET_H, *W2 = b1 + NET_H, *b2 = W2 + NET_H * NET_H,
                *W3 = b2 + NET_H, *b3 = W3 + NET_H * NET_H, *W4 = b3 + NET_H, *b4 = W4 + (size_t)NET_NV * NET_H;
    net->W1 = (float *)malloc(sizeof(float) * (size_t)NET_NV * NET_H);
    net->W2 = (float *)malloc(sizeof(float) * NET_H * NET_H);
    net->W3 = (float *)malloc(sizeof(float) * NET_H * NET_H);
    net->W4 = (float *)malloc(sizeof(float) * (size_t)NET_NV * NET_H);
    for (size_t k = 0; k < (size_t)NET_NV * NET_H; ++k) {
        net->W1[k] = bf16_round(W1[k]);
        net->W4[k] = bf16_round(W4[k]);
    }
    for (int k = 0; k < NET_H * NET_H; ++k) {
        net->W2[k] = bf16_round(W2[k]);
        net->W3[k] = bf16_round(W3[k]);
    }
    net->b1 = b1; net->b2 = b2; net->b3 = b3; net->b4 = b4;
}

static void net_release(orc_net *net)
{
    free(net->W1); free(net->W2); free(net->W3); free(net->W4);
}

/* Voxel (iz*16 + iy)*16 + ix of a point of the gas region, each axis cut in 16
 * equal cells, indices clamped to the grid. */
static int voxel_of(const orc_config *c, const double *p)
{
    long ix = (long)floor(p[0] * (NET_G / c->lx));
    long iy = (long)floor(p[1] * (NET_G / c->ly));
    long iz = (long)floor((p[2] - c->zlo) * (NET_G / (c->zhi - c->zlo)));
    ix = ix < 0 ? 0 : (ix > NET_G - 1 ? NET_G - 1 : ix);
    iy = iy < 0 ? 0 : (iy > NET_G - 1 ? NET_G - 1 : iy);
    iz = iz < 0 ? 0 : (iz > NET_G - 1 ? NET_G - 1 : iz);
    return (int)((iz * NET_G + iy) * NET_G + ix);
}

/* hidden layer: out[o] = bf16(gelu(sum_k W[o][k] in[k] + b[o])) */
static void net_layer(const float *W, const float *b, const float *in, float *out)
{
    for (int o = 0; o < NET_H; ++o) {
        float s = 0.0f;
        for (int k = 0; k < NET_H; ++k) s += W[o * NET_H + k] * in[k];
        out[o] = bf16_round(gelu(s + b[o]));
    }
}

/* Logits of the network for the occupancy of xyz[0..n) without particle `skip`
 * (-1: none); returns the log-normaliser ln sum_v exp(logit_v).  The first layer
 * is the sum over occupied voxels, in ascending voxel order, of count * W1 row. */
static double net_logits(const orc_config *c, const orc_net *net, const double *xyz, int n, int skip,
                         float *logit)
{
    int occ[NET_NV];
    memset(occ, 0, sizeof occ);
    for (int j = 0; j < n; ++j)
        if (j != skip) occ[voxel_of(c, xyz + 3 * j)]++;
    float a[NET_H], h1[NET_H], h2[NET_H], h3[NET_H];
    for (int k = 0; k < NET_H; ++k) a[k] = net->b1[k];
    for (int v = 0; v < NET_NV; ++v) {
        if (!occ[v]) continue;
        const float cnt = (float)occ[v];
        for (int k = 0; k < NET_H; ++k) a[k] += cnt * net->W1[(size_t)v * NET_H + k];
    }
    for (int k = 0; k < NET_H; ++k) h1[k] = bf16_round(gelu(a[k]));
    net_layer(net->W2, net->b2, h1, h2);
    net_layer(net->W3, net->b3, h2, h3);
    double mx = -INFINITY;
    for (int v = 0; v < NET_NV; ++v) {
        float s = 0.0f;
        for (int k = 0; k < NET_H; ++k) s += net->W4[(size_t)v * NET_H + k] * h3[k];
        logit[v] = s + net->b4[v];
        if ((double)logit[v] > mx) mx = (double)logit[v];
    }
    double sum = 0.0;
    for (int v = 0; v < NET_NV; ++v) sum += exp((double)logit[v] - mx);
    return mx + log(sum);
}

/* Gumbel-max draw from softmax(logit): the voxel maximising logit_v - ln(-ln u_v),
 * u_v = open uniform of word v%4 of the Philox block (t, sweep, walker, 16 + v/4);
 * ties go to the lowest v.  *gap = best key minus the runner-up. */
static int gumbel_argmax(const orc_config *c, const float *logit, uint32_t t, uint32_t sweep, uint32_t wid,
                         double *gap)
{
    double best = -INFINITY, second = -INFINITY;
    int arg = 0;
    for (int b = 0; b < NET_NV / 4; ++b) {
        uint32_t R[4];
        philox_words(c->seed, t, sweep, wid, 16u + (uint32_t)b, R);
        for (int q = 0; q < 4; ++q) {
            const int v = 4 * b + q;
            const double key = (double)logit[v] - log(-log(u32_open(R[q])));
            if (key > best) {
                second = best;
                best = key;
                arg = v;
            } else if (key > second) {
                second = key;
            }
        }
    }
    *gap = best - second;
    return arg;
}

/* ln q(r|X) - ln(1/V) = ln(1 + alpha (P_v V / V_vox - 1)), with V / V_vox = 4096 */
static double ln_q_ratio(double alpha, double lnp)
{
    return log1p(alpha * (exp(lnp) * (double)NET_NV - 1.0));
}

/* exported for the tests */
int orc_voxel_of(const orc_config *c, const double *p) { return voxel_of(c, p); }

double orc_net_logits(const orc_config *c, const double *xyz, int n, int skip, float *logit)
{
    orc_net net;
    net_prepare(c->net, &net);
    double lse = net_logits(c, &net, xyz, n, skip, logit);
    net_release(&net);
    return lse;
}

int orc_gumbel_argmax(const orc_config *c, const float *logit, uint32_t t, uint32_t sweep, uint32_t wid,
                      double *gap)
{
    return gumbel_argmax(c, logit, t, sweep, wid, gap);
}

/* ------------------------------------------------------------------------- */
/* Structural observables of one configuration                               */
/* ------------------------------------------------------------------------- */
int orc_obs_count(const orc_config *c)
{
    if (c->obs_dz <= 0.0) return 0;
    return (int)ceil((c->zhi - c->zlo) / c->obs_dz) + c->obs_nr + 1;
}

void orc_observables(const orc_config *c, const double *xyz, int n, double *out)
{
    if (c->obs_dz <= 0.0) return;     /* no observables configured (orc_obs_count is 0) */
    const int nz = (int)ceil((c->zhi - c->zlo) / c->obs_dz);
    const int no = nz + c->obs_nr + 1;
    for (int k = 0; k < no; ++k) out[k] = 0.0;
    int in_layer = 0;
    for (int i = 0; i < n; ++i) {
        const double z = xyz[3 * i + 2];
        int kz = (int)floor((z - c->zlo) / c->obs_dz);
        kz = kz < 0 ? 0 : (kz > nz - 1 ? nz - 1 : kz);
        out[kz] += 1.0;
        if (z >= c->obs_layer_lo && z < c->obs_layer_hi) ++in_layer;
    }
    for (int i = 0; i < n; ++i) {
        const double zi = xyz[3 * i + 2];
        if (!(zi >= c->obs_layer_lo && zi < c->obs_layer_hi)) continue;
        for (int j = i + 1; j < n; ++j) {
            const double zj = xyz[3 * j + 2];
            if (!(zj >= c->obs_layer_lo && zj < c->obs_layer_hi)) continue;
            const double dx = min_image(xyz[3 * i] - xyz[3 * j], c->lx);
            const double dy = min_image(xyz[3 * i + 1] - xyz[3 * j + 1], c->ly);
            const double r = sqrt(dx * dx + dy * dy);
            const int kr = (int)floor(r / c->obs_dr);
            if (kr < c->obs_nr) out[nz + kr] += 1.0;
        }
    }
    out[nz + c->obs_nr] = (double)in_layer;
}

/* ------------------------------------------------------------------------- */
/* One trial move of one walker                                              */
/* ------------------------------------------------------------------------- */
typedef struct {
    int32_t *n;        /* [S] */
    double *e;         /* [S] */
    int32_t *label;    /* [S] state held by walker */
    int32_t *wos;      /* [S] walker holding state */
    double *xyz;       /* [S][n_max][3] */
    int32_t *site;     /* [S][n_max] site index (mode 2), may be NULL otherwise */
    int64_t *stats;    /* [S][ORC_NSTAT] by state */
    int64_t *swap_att; /* [4][S] by swap type and lower state of the pair */
    int64_t *swap_acc;
    /* [n_sweeps][S][K] or NULL: per trial, the distance of the learned proposal's
     * decisions from their thresholds (|ln A - ln U|, and the Gumbel-max gap of a
     * network-drawn voxel); +inf for trials the network took no part in */
    float *margin;
    /* [samples][n_obs] or NULL: the observables of every recorded sample */
    double *obs;
    /* lowest-energy recorded configuration of each N (Sec. III.A, aiAT@REGC step
     * (i)), or NULL: min_e [n_max+1] (+inf where N was never recorded), min_xyz
     * [n_max+1][n_max][3]; updated at every sample point, walkers in index order,
     * replaced only by a strictly lower energy */
    double *min_e, *min_xyz;
    /* molecular dynamics: velocities [S][n_max][3] and the temperature they were
     * drawn or last thermalised at, per walker (0: not initialised) */
    double *vel, *tv;
} orc_walkers;

/* Metropolis decision on x = ln(acceptance ratio): accept when x >= 0, else
 * when the uniform U is below exp(x). */
static int metropolis(double x, double U)
{
    if (x >= 0.0) return 1;
    return U < exp(x);
}

static int site_occupied(const int32_t *site, int n, int k)
{
    for (int j = 0; j < n; ++j)
        if (site[j] == k) return 1;
    return 0;
}

/* Returns 1 if the trial was accepted.  `lnk` holds log(k) for k = 0..n_max+1. */
/* kind: -1 draws the move type from A0 with p_disp and p_ins; -2 draws a particle
 * exchange (removal when A0 / 2^32 < 1/2, else insertion); 0 displacement,
 * 1 insertion, 2 removal force it. */
static int trial(const orc_config *c, const orc_statec *sc, const double *lnk, double lnv,
                 const orc_net *net, orc_walkers *W, int w, int64_t sweep, int t, float *margin, int kind)
{
    uint32_t A[4], B[4];
    const uint32_t wid = (uint32_t)(w + c->walker_offset);
    philox_words(c->seed, (uint32_t)t, (uint32_t)sweep, wid, 0u, A);
    philox_words(c->seed, (uint32_t)t, (uint32_t)sweep, wid, 1u, B);

    const int s = W->label[w];
    const double beta = sc[s].beta, lnz = sc[s].lnz;
    int64_t *st = W->stats + (int64_t)s * ORC_NSTAT;
    int n = W->n[w];
    double *xyz = W->xyz + (int64_t)w * c->n_max * 3;
    int32_t *site = W->site ? W->site + (int64_t)w * c->n_max : NULL;
    const double U = u53(B[1], B[2]);

    const uint64_t th_disp = (uint64_t)llround(c->p_disp * 4294967296.0);
    const uint64_t th_ins = th_disp + (uint64_t)llround(c->p_ins * 4294967296.0);
    const uint64_t a0 = A[0];
    const int k = kind >= 0 ? kind
                            : (kind == -2 ? (a0 < 0x80000000u ? 2 : 1) : (a0 < th_disp ? 0 : (a0 < th_ins ? 1 : 2)));

    if (k == 0) {
        /* ---- displacement, Eq. (7) ---- */
        st[ST_DISP_ATT]++;
        if (n == 0) { st[ST_EMPTY_REJ]++; return 0; }
        int i = (int)(((uint64_t)A[1] * (uint64_t)n) >> 32);
        double *ri = xyz + 3 * i;
        double de;
        double p[3];
        int core_new = 0, core_old = 0;
        if (c->mode == 2) {
            int k = (int)(((uint64_t)A[2] * (uint64_t)c->n_sites) >> 32);
            if (site_occupied(site, n, k)) { return 0; }
            memcpy(p, c->sites + 3 * k, sizeof p);
            double e_new = particle_energy(c, p, xyz, n, i, &core_new);
            double e_old = particle_energy(c, ri, xyz, n, i, &core_old);
            de = e_new - e_old;
            double x = -beta * de;
            if (metropolis(x, U)) {
                memcpy(ri, p, sizeof p);
                site[i] = k;
                W->e[w] += de;
                st[ST_DISP_ACC]++;
                return 1;
            }
            return 0;
        }
        double d = c->max_disp;
        p[0] = ri[0] + d * (2.0 * u32_open(A[2]) - 1.0);
        p[1] = ri[1] + d * (2.0 * u32_open(A[3]) - 1.0);
        p[2] = ri[2] + d * (2.0 * u32_open(B[0]) - 1.0);
        if (p[0] < 0.0) p[0] += c->lx; else if (p[0] >= c->lx) p[0] -= c->lx;
        if (p[1] < 0.0) p[1] += c->ly; else if (p[1] >= c->ly) p[1] -= c->ly;
        if (p[2] < c->zlo || p[2] > c->zhi) { st[ST_WALL_REJ]++; return 0; }
        if (c->mode == 1) {
            de = 0.0;
        } else {
            double e_new = particle_energy(c, p, xyz, n, i, &core_new);
            if (core_new) { st[ST_CORE_REJ]++; return 0; }
            double e_old = particle_energy(c, ri, xyz, n, i, &core_old);
            de = e_new - e_old;
        }
        double x = -beta * de;
        if (metropolis(x, U)) {
            memcpy(ri, p, sizeof p);
            W->e[w] += de;
            st[ST_DISP_ACC]++;
            return 1;
        }
        return 0;
    } else if (k == 1) {
        /* ---- insertion, Eq. (3) with the corrected exponent ---- */
        st[ST_INS_ATT]++;
        if (n >= c->n_max) { st[ST_CAP_REJ]++; return 0; }
        double p[3];
        int core = 0, k = -1;
        double lnq = 0.0;
        if (c->mode == 2) {
            k = (int)(((uint64_t)A[2] * (uint64_t)c->n_sites) >> 32);
            if (site_occupied(site, n, k)) return 0;
            memcpy(p, c->sites + 3 * k, sizeof p);
        } else if (net) {
            /* learned proposal: network voxel with probability alpha, else uniform */
            float logit[NET_NV];
            const double lse = net_logits(c, net, xyz, n, -1, logit);
            int v;
            if (u32_open(B[3]) < c->alpha) {
                double gap;
                v = gumbel_argmax(c, logit, (uint32_t)t, (uint32_t)sweep, wid, &gap);
                if (margin) *margin = (float)gap;
                const int ix = v % NET_G, iy = (v / NET_G) % NET_G, iz = v / (NET_G * NET_G);
                p[0] = ((double)ix + u32_open(A[2])) * (c->lx / NET_G);
                p[1] = ((double)iy + u32_open(A[3])) * (c->ly / NET_G);
                p[2] = c->zlo + ((double)iz + u32_open(B[0])) * ((c->zhi - c->zlo) / NET_G);
                /* a point rounded onto a neighbouring voxel is not a draw of v */
                if (voxel_of(c, p) != v) { st[ST_WALL_REJ]++; return 0; }
            } else {
                p[0] = c->lx * u32_open(A[2]);
                p[1] = c->ly * u32_open(A[3]);
                p[2] = c->zlo + (c->zhi - c->zlo) * u32_open(B[0]);
                v = voxel_of(c, p);
            }
            lnq = ln_q_ratio(c->alpha, (double)logit[v] - lse);
        } else {
            p[0] = c->lx * u32_open(A[2]);
            p[1] = c->ly * u32_open(A[3]);
            p[2] = c->zlo + (c->zhi - c->zlo) * u32_open(B[0]);
        }
        double de = 0.0;
        if (c->mode != 1) {
            de = particle_energy(c, p, xyz, n, -1, &core);
            if (core && c->mode == 0) { st[ST_CORE_REJ]++; return 0; }
        }
        /* ln A = ln z + ln V - ln(N+1) - beta dE  (V -> number of sites in mode 2);
         * learned proposal: ln V -> -ln q = ln V - lnq */
        double x = (((lnz + lnv) - lnk[n + 1]) - lnq) - beta * de;
        if (net && margin) {
            const float mg = (float)fabs(x - log(U));
            if (mg < *margin) *margin = mg;
        }
        if (metropolis(x, U)) {
            memcpy(xyz + 3 * n, p, sizeof p);
            if (site) site[n] = k;
            W->n[w] = n + 1;
            W->e[w] += de;
            st[ST_INS_ACC]++;
            return 1;
        }
        return 0;
    } else {
        /* ---- removal, Eq. (2) ---- */
        st[ST_DEL_ATT]++;
        if (n == 0) { st[ST_EMPTY_REJ]++; return 0; }
        int i = (int)(((uint64_t)A[1] * (uint64_t)n) >> 32);
        double de = 0.0;
        int core = 0;
        if (c->mode != 1) de = -particle_energy(c, xyz + 3 * i, xyz, n, i, &core);
        /* learned proposal: the reverse insertion's density at r_i, on the occupancy
         * of the configuration without i */
        double lnq = 0.0;
        if (net) {
            float logit[NET_NV];
            const double lse = net_logits(c, net, xyz, n, i, logit);
            lnq = ln_q_ratio(c->alpha, (double)logit[voxel_of(c, xyz + 3 * i)] - lse);
        }
        /* ln A = ln N - ln z - ln V - beta dE,  dE = E_{N-1} - E_N;
         * learned proposal: -ln V -> ln q = -ln V + lnq */
        double x = ((lnk[n] - (lnz + lnv)) + lnq) - beta * de;
        if (net && margin) {
            const float mg = (float)fabs(x - log(U));
            if (mg < *margin) *margin = mg;
        }
        if (metropolis(x, U)) {
            /* the removed slot is refilled by the last particle */
            if (i != n - 1) {
                memcpy(xyz + 3 * i, xyz + 3 * (n - 1), 3 * sizeof(double));
                if (site) site[i] = site[n - 1];
            }
            W->n[w] = n - 1;
            W->e[w] += de;
            st[ST_DEL_ACC]++;
            return 1;
        }
        return 0;
    }
}

/* ------------------------------------------------------------------------- */
/* Replica-exchange step                                                     */
/* ------------------------------------------------------------------------- */
/* Collective neighbour swaps (Sec. II.A.2).  One of four pair types is drawn
 * with probability 1/4; all its disjoint pairs are attempted independently.
 *   scheme 0: type 0 T-pairs (2a,2a+1), type 1 T-pairs (2a+1,2a+2),
 *             type 2 mu-pairs (2b,2b+1), type 3 mu-pairs (2b+1,2b+2).
 *   scheme 1: within 2x2 blocks: type 0 along T, type 1 along mu,
 *             type 2 main diagonal, type 3 anti-diagonal; the blocks start at
 *             (ol + 2a, om + 2b) with ol, om drawn per step (bits 29, 28 of the
 *             type word), so blocks of the even and odd tilings alternate.
 * Pair acceptance from Eq. (1) of both walkers in both states. */
static void swap_pair(const orc_config *c, const orc_statec *sc, orc_walkers *W, int64_t q,
                      int type, int sa, int sb)
{
    int S = c->n_t * c->n_mu;
    int lo = sa < sb ? sa : sb;
    uint32_t R[4];
    philox_words(c->seed, (uint32_t)lo, (uint32_t)q, 0xFFFFFFFFu - (uint32_t)c->class_id, 4u, R);
    int i = W->wos[sa], j = W->wos[sb];
    double x = (sc[sa].beta - sc[sb].beta) * (W->e[i] - W->e[j])
             + (double)(W->n[j] - W->n[i]) * (sc[sa].lnz - sc[sb].lnz);
    W->swap_att[(int64_t)type * S + lo]++;
    if (metropolis(x, u53(R[0], R[1]))) {
        W->label[i] = sb;
        W->label[j] = sa;
        W->wos[sa] = j;
        W->wos[sb] = i;
        W->swap_acc[(int64_t)type * S + lo]++;
    }
}

static void swap_step(const orc_config *c, const orc_statec *sc, orc_walkers *W, int64_t q)
{
    uint32_t R[4];
    philox_words(c->seed, 0u, (uint32_t)q, 0xFFFFFFFFu - (uint32_t)c->class_id, 3u, R);
    int type = (int)(R[0] >> 30);
    int L = c->n_t, M = c->n_mu;
    if (c->swap_scheme == 0) {
        if (type < 2) {
            for (int l = type; l + 1 < L; l += 2)
                for (int m = 0; m < M; ++m) swap_pair(c, sc, W, q, type, l * M + m, (l + 1) * M + m);
        } else {
            for (int l = 0; l < L; ++l)
                for (int m = type - 2; m + 1 < M; m += 2) swap_pair(c, sc, W, q, type, l * M + m, l * M + m + 1);
        }
    } else {
        /* block origin (ol, om) in {0,1}^2 from the next two bits of the type word:
         * the 2x2 blocks alternate between the even and odd tilings of each axis,
         * so a configuration can leave the block it started in */
        int ol = (int)((R[0] >> 29) & 1u), om = (int)((R[0] >> 28) & 1u);
        for (int l = ol; l + 1 < L; l += 2) {
            for (int m = om; m + 1 < M; m += 2) {
                int s00 = l * M + m, s01 = l * M + m + 1, s10 = (l + 1) * M + m, s11 = (l + 1) * M + m + 1;
                if (type == 0) { swap_pair(c, sc, W, q, type, s00, s10); swap_pair(c, sc, W, q, type, s01, s11); }
                if (type == 1) { swap_pair(c, sc, W, q, type, s00, s01); swap_pair(c, sc, W, q, type, s10, s11); }
                if (type == 2) { swap_pair(c, sc, W, q, type, s00, s11); }
                if (type == 3) { swap_pair(c, sc, W, q, type, s01, s10); }
            }
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Molecular dynamics for the canonical part of the REGC step               */
/* ------------------------------------------------------------------------- */
/* Standard normals by Box-Muller from two open uniforms:
 * sqrt(-2 ln u1) cos(2 pi u2), sqrt(-2 ln u1) sin(2 pi u2). */
static void box_muller(uint32_t w1, uint32_t w2, double *z0, double *z1)
{
    const double r = sqrt(-2.0 * log(u32_open(w1)));
    const double a = 6.283185307179586 * u32_open(w2);
    *z0 = r * cos(a);
    *z1 = r * sin(a);
}

/* three normals of Philox block (t, q, walker, tag): words (0,1) and (2,3) */
static void normals3(const orc_config *c, uint32_t t, uint32_t q, uint32_t wid, uint32_t tag, double z[3])
{
    uint32_t R[4];
    double unused;
    philox_words(c->seed, t, q, wid, tag, R);
    box_muller(R[0], R[1], &z[0], &z[1]);
    box_muller(R[2], R[3], &z[2], &unused);
}

/* Forces (negative gradient of the truncated-shifted LJ energy; the shift does not
 * act) on every gas particle from the other gas particles and the slab, and the
 * potential energy E = sum over gas pairs + gas-slab pairs.  Particle i sums its
 * partners in order: gas j = 0..n-1 (j != i), then the slab atoms in input order. */
static double md_forces(const orc_config *c, const double *xyz, int n, double *f)
{
    const double rc2 = c->rc * c->rc;
    double e = 0.0;
    for (int i = 0; i < n; ++i) {
        double fx = 0.0, fy = 0.0, fz = 0.0, ei = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            const double dx = min_image(xyz[3 * i] - xyz[3 * j], c->lx);
            const double dy = min_image(xyz[3 * i + 1] - xyz[3 * j + 1], c->ly);
            const double dz = xyz[3 * i + 2] - xyz[3 * j + 2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 >= rc2) continue;
            const double s2 = (c->sig_gg * c->sig_gg) / r2, s6 = s2 * s2 * s2;
            const double g = 24.0 * c->eps_gg * (2.0 * s6 * s6 - s6) / r2;     /* -phi'(r)/r */
            fx += g * dx; fy += g * dy; fz += g * dz;
            ei += 0.5 * orc_lj(r2, c->eps_gg, c->sig_gg, c->rc, c->shifted);
        }
        for (int a = 0; a < c->n_slab; ++a) {
            const double *sa = c->slab + 3 * a;
            const double dx = min_image(xyz[3 * i] - sa[0], c->lx);
            const double dy = min_image(xyz[3 * i + 1] - sa[1], c->ly);
            const double dz = xyz[3 * i + 2] - sa[2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 >= rc2) continue;
            const double s2 = (c->sig_gs * c->sig_gs) / r2, s6 = s2 * s2 * s2;
            const double g = 24.0 * c->eps_gs * (2.0 * s6 * s6 - s6) / r2;
            fx += g * dx; fy += g * dy; fz += g * dz;
            ei += orc_lj(r2, c->eps_gs, c->sig_gs, c->rc, c->shifted);
        }
        f[3 * i] = fx; f[3 * i + 1] = fy; f[3 * i + 2] = fz;
        e += ei;
    }
    return e;
}

double orc_md_forces(const orc_config *c, const double *xyz, int n, double *f) { return md_forces(c, xyz, n, f); }

/* Stochastic velocity rescaling (Bussi, Donadio, Parrinello, J. Chem. Phys. 126,
 * 014101 (2007)): the kinetic energy K of Nf = 3N degrees of freedom is moved to
 *   K' = c K + (1 - c) Kbar (R1^2 + S)/Nf + 2 sqrt(c (1 - c) K Kbar / Nf) R1,
 * c = exp(-dt/tau), Kbar = Nf kT / 2, R1 a standard normal, S the sum of Nf - 1
 * squared standard normals; velocities scale by sqrt(K'/K).  R1: word pair (0,1)
 * of Philox block (t, q, walker, 2); S: the normals of blocks (t, q, walker, 16 + b),
 * four per block (Box-Muller on word pairs (0,1), (2,3)), the first Nf - 1 of them. */
static void md_thermostat(const orc_config *c, double *v, int n, double T, uint32_t t, uint32_t q, uint32_t wid)
{
    const int nf = 3 * n;
    double K = 0.0;
    for (int k = 0; k < nf; ++k) K += 0.5 * v[k] * v[k];
    if (!(K > 0.0)) return;
    const double Kbar = 0.5 * nf * T;
    const double cc = exp(-c->md_dt / c->md_tau);
    uint32_t R[4];
    double r1, unused;
    philox_words(c->seed, t, q, wid, 2u, R);
    box_muller(R[0], R[1], &r1, &unused);
    double S = 0.0;
    for (int b = 0; 4 * b < nf - 1; ++b) {
        double z[4];
        philox_words(c->seed, t, q, wid, 16u + (uint32_t)b, R);
        box_muller(R[0], R[1], &z[0], &z[1]);
        box_muller(R[2], R[3], &z[2], &z[3]);
        for (int k = 0; k < 4 && 4 * b + k < nf - 1; ++k) S += z[k] * z[k];
    }
    const double K2 = cc * K + (1.0 - cc) * Kbar * (r1 * r1 + S) / nf + 2.0 * sqrt(cc * (1.0 - cc) * K * Kbar / nf) * r1;
    const double alpha = sqrt(K2 / K);
    for (int k = 0; k < nf; ++k) v[k] *= alpha;
}

/* md_steps velocity-Verlet steps of walker w in REGC step q (forces at the start
 * recomputed, positions wrapped in x, y and reflected at the walls in z); the
 * running energy becomes the potential energy of the final configuration. */
static void md_run(const orc_config *c, const orc_statec *sc, orc_walkers *W, int w, int64_t q)
{
    const int n = W->n[w];
    if (n == 0) return;
    const double T = 1.0 / sc[W->label[w]].beta, dt = c->md_dt;
    const uint32_t wid = (uint32_t)(w + c->walker_offset);
    double *x = W->xyz + (int64_t)w * c->n_max * 3, *v = W->vel + (int64_t)w * c->n_max * 3;
    double *f = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double e = md_forces(c, x, n, f);
    for (int st = 0; st < c->md_steps; ++st) {
        for (int k = 0; k < 3 * n; ++k) v[k] += 0.5 * dt * f[k];
        for (int i = 0; i < n; ++i) {
            double *p = x + 3 * i, *u = v + 3 * i;
            p[0] += dt * u[0]; p[1] += dt * u[1]; p[2] += dt * u[2];
            if (p[0] < 0.0) p[0] += c->lx; else if (p[0] >= c->lx) p[0] -= c->lx;
            if (p[1] < 0.0) p[1] += c->ly; else if (p[1] >= c->ly) p[1] -= c->ly;
            if (p[2] < c->zlo) { p[2] = 2.0 * c->zlo - p[2]; u[2] = -u[2]; }
            else if (p[2] > c->zhi) { p[2] = 2.0 * c->zhi - p[2]; u[2] = -u[2]; }
        }
        e = md_forces(c, x, n, f);
        for (int k = 0; k < 3 * n; ++k) v[k] += 0.5 * dt * f[k];
        if (c->md_tau > 0.0) md_thermostat(c, v, n, T, (uint32_t)(1 + st), (uint32_t)q, wid);
    }
    W->e[w] = e;
    free(f);
}

/* Before the exchange attempt of step q: velocities of a walker not initialised
 * are drawn from the Maxwell-Boltzmann law at its state's T (particle i: normals of
 * block (0x80000000 + i, q, walker, 4)); a walker whose state T changed since (an
 * exchange) has its velocities scaled by sqrt(T_new / T_old). */
static void md_prepare(const orc_config *c, const orc_statec *sc, orc_walkers *W, int w, int64_t q)
{
    const double T = 1.0 / sc[W->label[w]].beta;
    const uint32_t wid = (uint32_t)(w + c->walker_offset);
    double *v = W->vel + (int64_t)w * c->n_max * 3;
    if (W->tv[w] == 0.0) {
        for (int i = 0; i < W->n[w]; ++i) {
            double z[3];
            normals3(c, 0x80000000u + (uint32_t)i, (uint32_t)q, wid, 4u, z);
            for (int k = 0; k < 3; ++k) v[3 * i + k] = sqrt(T) * z[k];
        }
    } else if (W->tv[w] != T) {
        const double s = sqrt(T / W->tv[w]);
        for (int k = 0; k < 3 * W->n[w]; ++k) v[k] *= s;
    }
    W->tv[w] = T;
}

/* ------------------------------------------------------------------------- */
/* The paper's REGC step (Sec. II.A, Sec. III.A)                             */
/* ------------------------------------------------------------------------- */
/* Step q: a coin from Philox (0, q, 0xFFFFFFFF - class, 6), open uniform of word 0,
 * below x0 -> every walker attempts one particle exchange with the reservoir
 * (trial 0: removal or insertion with probability 1/2), otherwise the replica-
 * exchange step q of the same four collective types.  Then every walker runs
 * mc_cycles MC cycles of N displacement attempts (trials 1 .. mc_cycles N, N after
 * the exchange attempt).  Samples after the step when (q+1) % sample_every == 0.
 * Trace rows hold ceil((1 + mc_cycles n_max)/32) words per walker and step. */
static int run_paper_schedule(const orc_config *c, const orc_statec *sc, const double *lnk, double lnv,
                              const orc_net *net, orc_walkers *W, int64_t *step, int64_t n_steps, double *samp_e,
                              int32_t *samp_n, int32_t *samp_s, int64_t samp_cap, int64_t *samp_count,
                              uint32_t *trace_bits, int32_t *trace_n, int n_threads)
{
    const int S = c->n_t * c->n_mu;
    const int Kmax = 1 + c->mc_cycles * c->n_max;
    const int words = (Kmax + 31) / 32;
    for (int64_t it = 0; it < n_steps; ++it) {
        const int64_t q = *step;
        if (c->sample_every > 0 && (q + 1) % c->sample_every == 0 && *samp_count + S > samp_cap) return -4;
        uint32_t R[4];
        philox_words(c->seed, 0u, (uint32_t)q, 0xFFFFFFFFu - (uint32_t)c->class_id, 6u, R);
        const int gc = u32_open(R[0]) < c->x0;
        if (!gc) swap_step(c, sc, W, q);
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads)
        for (int w = 0; w < S; ++w) {
            uint32_t *bits = trace_bits ? trace_bits + ((int64_t)it * S + w) * words : NULL;
            float *mrow = W->margin ? W->margin + ((int64_t)it * S + w) * Kmax : NULL;
            if (bits) memset(bits, 0, sizeof(uint32_t) * words);
            if (mrow)
                for (int t = 0; t < Kmax; ++t) mrow[t] = INFINITY;
            const int md = c->md_steps > 0;
            if (md) md_prepare(c, sc, W, w, q);
            const int n_before = W->n[w];
            if (gc && trial(c, sc, lnk, lnv, net, W, w, q, 0, mrow, -2) && bits) bits[0] |= 1u;
            if (md) {
                /* the inserted particle gets Maxwell-Boltzmann velocities (block (0, q,
                 * walker, 3)); the removed slot takes the last particle's velocity */
                double *v = W->vel + (int64_t)w * c->n_max * 3;
                const uint32_t wid = (uint32_t)(w + c->walker_offset);
                if (W->n[w] > n_before) {
                    double z[3];
                    normals3(c, 0u, (uint32_t)q, wid, 3u, z);
                    const double T = 1.0 / sc[W->label[w]].beta;
                    for (int k = 0; k < 3; ++k) v[3 * n_before + k] = sqrt(T) * z[k];
                } else if (W->n[w] < n_before) {
                    uint32_t A[4];
                    philox_words(c->seed, 0u, (uint32_t)q, wid, 0u, A);
                    const int i = (int)(((uint64_t)A[1] * (uint64_t)n_before) >> 32);
                    if (i != n_before - 1) memcpy(v + 3 * i, v + 3 * (n_before - 1), 3 * sizeof(double));
                }
                md_run(c, sc, W, w, q);
            } else {
                const int T = 1 + c->mc_cycles * W->n[w];
                for (int t = 1; t < T; ++t) {
                    int acc = trial(c, sc, lnk, lnv, net, W, w, q, t, mrow ? mrow + t : NULL, 0);
                    if (bits && acc) bits[t >> 5] |= 1u << (t & 31);
                }
            }
            if (trace_n) trace_n[(int64_t)it * S + w] = W->n[w];
        }
        if (c->sample_every > 0 && (q + 1) % c->sample_every == 0) {
            for (int w = 0; w < S; ++w) {
                if (W->min_e && W->e[w] < W->min_e[W->n[w]]) {
                    W->min_e[W->n[w]] = W->e[w];
                    memcpy(W->min_xyz + (int64_t)W->n[w] * c->n_max * 3, W->xyz + (int64_t)w * c->n_max * 3,
                           sizeof(double) * 3 * (size_t)W->n[w]);
                }
                if (W->obs && c->obs_dz > 0.0)
                    orc_observables(c, W->xyz + (int64_t)w * c->n_max * 3, W->n[w],
                                    W->obs + *samp_count * orc_obs_count(c));
                samp_e[*samp_count] = W->e[w];
                samp_n[*samp_count] = W->n[w];
                samp_s[*samp_count] = W->label[w];
                (*samp_count)++;
            }
        }
        *step = q + 1;
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Driver                                                                    */
/* ------------------------------------------------------------------------- */
/* Runs sweeps [*sweep, *sweep + n_sweeps) of the whole REGC simulation.
 * After every sweep s: samples (E, N, state) of all walkers are appended when
 * (s+1) % sample_every == 0; then the replica-exchange step q = (s+1)/swap_every - 1
 * runs when (s+1) % swap_every == 0.
 * trace_bits: [n_sweeps][S][ceil(K/32)] accept bits (may be NULL);
 * trace_n:    [n_sweeps][S] N at each sweep end (may be NULL).
 * Returns 0, or -4 when the sample buffer is too small (nothing is lost: the
 * run stops before the sweep whose samples would not fit).
 * With schedule 1 the unit is the paper's REGC step instead of the sweep
 * (run_paper_schedule). */
int orc_run(const orc_config *c, orc_walkers *W, int64_t *sweep, int64_t n_sweeps,
            double *samp_e, int32_t *samp_n, int32_t *samp_s, int64_t samp_cap, int64_t *samp_count,
            uint32_t *trace_bits, int32_t *trace_n, int n_threads)
{
    const int S = c->n_t * c->n_mu;
    const int K = c->trials_per_sweep > 0 ? c->trials_per_sweep : c->n_max + 1;
    const int words = (K + 31) / 32;
    orc_statec *sc = (orc_statec *)malloc(sizeof(orc_statec) * S);
    double *lnk = (double *)malloc(sizeof(double) * (c->n_max + 2));
    state_constants(c, sc);
    lnk[0] = 0.0;
    for (int k = 1; k <= c->n_max + 1; ++k) lnk[k] = log((double)k);
    double lnv = (c->mode == 2) ? log((double)c->n_sites)
                                : log(c->lx * c->ly * (c->zhi - c->zlo));
    int rc = 0;
    /* the network takes part only with alpha > 0 (alpha = 0 is the plain method) */
    orc_net netr, *net = NULL;
    if (c->net && c->alpha > 0.0) {
        if (c->mode == 2 || c->alpha > 1.0) {
            free(sc);
            free(lnk);
            return -6;
        }
        net_prepare(c->net, &netr);
        net = &netr;
    }
    if (c->schedule == 1) {
        rc = run_paper_schedule(c, sc, lnk, lnv, net, W, sweep, n_sweeps, samp_e, samp_n, samp_s, samp_cap,
                                samp_count, trace_bits, trace_n, n_threads);
        n_sweeps = 0;
    }
    for (int64_t it = 0; it < n_sweeps; ++it) {
        const int64_t s = *sweep;
        if (c->sample_every > 0 && (s + 1) % c->sample_every == 0 && *samp_count + S > samp_cap) {
            rc = -4;
            break;
        }
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads)
        for (int w = 0; w < S; ++w) {
            uint32_t *bits = trace_bits ? trace_bits + ((int64_t)it * S + w) * words : NULL;
            float *mrow = W->margin ? W->margin + ((int64_t)it * S + w) * K : NULL;
            if (bits) memset(bits, 0, sizeof(uint32_t) * words);
            for (int t = 0; t < K; ++t) {
                if (mrow) mrow[t] = INFINITY;
                int acc = trial(c, sc, lnk, lnv, net, W, w, s, t, mrow ? mrow + t : NULL, -1);
                if (bits && acc) bits[t >> 5] |= 1u << (t & 31);
            }
            if (trace_n) trace_n[(int64_t)it * S + w] = W->n[w];
        }
        if (c->sample_every > 0 && (s + 1) % c->sample_every == 0) {
            for (int w = 0; w < S; ++w) {
                if (W->min_e && W->e[w] < W->min_e[W->n[w]]) {
                    W->min_e[W->n[w]] = W->e[w];
                    memcpy(W->min_xyz + (int64_t)W->n[w] * c->n_max * 3, W->xyz + (int64_t)w * c->n_max * 3,
                           sizeof(double) * 3 * (size_t)W->n[w]);
                }
                if (W->obs && c->obs_dz > 0.0)
                    orc_observables(c, W->xyz + (int64_t)w * c->n_max * 3, W->n[w],
                                    W->obs + *samp_count * orc_obs_count(c));
                samp_e[*samp_count] = W->e[w];
                samp_n[*samp_count] = W->n[w];
                samp_s[*samp_count] = W->label[w];
                (*samp_count)++;
            }
        }
        if (c->swap_every > 0 && (s + 1) % c->swap_every == 0)
            swap_step(c, sc, W, (s + 1) / c->swap_every - 1);
        *sweep = s + 1;
    }
    if (net) net_release(net);
    free(sc);
    free(lnk);
    return rc;
}

/* Single replica-exchange step, exposed for the detailed-balance tests. */
void orc_swap_step(const orc_config *c, orc_walkers *W, int64_t q)
{
    int S = c->n_t * c->n_mu;
    orc_statec *sc = (orc_statec *)malloc(sizeof(orc_statec) * S);
    state_constants(c, sc);
    swap_step(c, sc, W, q);
    free(sc);
}

/* ln of the swap acceptance ratio for walker i (in state a) and walker j (in state b). */
double orc_swap_lnratio(double beta_a, double lnz_a, double beta_b, double lnz_b,
                        double e_i, int n_i, double e_j, int n_j)
{
    return (beta_a - beta_b) * (e_i - e_j) + (double)(n_j - n_i) * (lnz_a - lnz_b);
}

/* aiAT@REGC phase map (Sec. III.A, Eq. (12)): with the free energies of the phases
 * approximated by their lowest sampled energies, dG_N(mu) = E_min(N) - E_min(0) - N mu
 * (the frozen slab has no energy of its own); the phase at mu is the N of lowest
 * dG among the recorded N (smallest N on ties).  phase [n_mu]. */
void orc_aiat_phase(int n_max, const double *min_e, int n_mu, const double *mu, int32_t *phase)
{
    for (int m = 0; m < n_mu; ++m) {
        double best = INFINITY;
        int arg = -1;
        for (int N = 0; N <= n_max; ++N) {
            if (!(min_e[N] < INFINITY)) continue;
            const double g = min_e[N] - (min_e[0] < INFINITY ? min_e[0] : 0.0) - (double)N * mu[m];
            if (g < best) {
                best = g;
                arg = N;
            }
        }
        phase[m] = arg;
    }
}


/* ------------------------------------------------------------------------- */
/* Checkpoint of a single-class simulation                                   */
/* ------------------------------------------------------------------------- */
/* The sampling state between two sweeps is (sweep counter, per walker N, running
 * energy, label, coordinates; walker-of-state table; per-state counters; exchange
 * counters): continuing from it repeats the uninterrupted chain exactly, since every
 * random number is keyed by (trial, sweep, walker).  Byte layout, little endian,
 * shared with the HIP library's checkpoint so that a blob moves between the two:
 *   u64 magic 0x3143474552, u32 version 1, u32 W, u32 n_max, u32 n_class (1),
 *   i64 sweep, u64 seed;
 *   i32 n[W], f64 e[W], i32 label[W], i32 wos[W], f64 xyz[W][n_max][3],
 *   i64 stats[W][10], i64 swap_att[4][W], i64 swap_acc[4][W].
 * Rows of xyz beyond a walker's N carry no state. */
#define ORC_CKPT_MAGIC 0x3143474552ULL
#define ORC_CKPT_HEADER 40

size_t orc_checkpoint_size(const orc_config *c)
{
    const size_t S = (size_t)c->n_t * (size_t)c->n_mu;
    return ORC_CKPT_HEADER + S * (4 + 8 + 4 + 4) + S * (size_t)c->n_max * 3 * 8 + S * ORC_NSTAT * 8 + 2 * 4 * S * 8;
}

static char *put(char *p, const void *src, size_t bytes)
{
    memcpy(p, src, bytes);
    return p + bytes;
}

/* Writes the checkpoint into buf (cap bytes).  Returns 0, or -4 when it does not fit. */
int orc_checkpoint(const orc_config *c, const orc_walkers *W, int64_t sweep, void *buf, size_t cap)
{
    const size_t S = (size_t)c->n_t * (size_t)c->n_mu;
    if (cap < orc_checkpoint_size(c)) return -4;
    uint64_t magic = ORC_CKPT_MAGIC, seed = c->seed;
    uint32_t version = 1, w32 = (uint32_t)S, nmax = (uint32_t)c->n_max, ncls = 1;
    char *p = (char *)buf;
    p = put(p, &magic, 8);
    p = put(p, &version, 4);
    p = put(p, &w32, 4);
    p = put(p, &nmax, 4);
    p = put(p, &ncls, 4);
    p = put(p, &sweep, 8);
    p = put(p, &seed, 8);
    p = put(p, W->n, S * 4);
    p = put(p, W->e, S * 8);
    p = put(p, W->label, S * 4);
    p = put(p, W->wos, S * 4);
    p = put(p, W->xyz, S * (size_t)c->n_max * 3 * 8);
    p = put(p, W->stats, S * ORC_NSTAT * 8);
    p = put(p, W->swap_att, 4 * S * 8);
    put(p, W->swap_acc, 4 * S * 8);
    return 0;
}

/* Restores a checkpoint written by orc_checkpoint (or by the HIP library for a
 * context of the same single class).  Nothing changes unless the blob matches this
 * configuration (size, magic, version, W, n_max, one class, seed), every N lies in
 * 0..n_max and the labels are a permutation whose inverse is the walker-of-state
 * table.  Returns 0 or -1. */
int orc_restore(const orc_config *c, orc_walkers *W, int64_t *sweep, const void *buf, size_t size)
{
    const size_t S = (size_t)c->n_t * (size_t)c->n_mu;
    if (size != orc_checkpoint_size(c)) return -1;
    const char *p = (const char *)buf;
    uint64_t magic, seed;
    uint32_t version, w32, nmax, ncls;
    int64_t sw;
    memcpy(&magic, p, 8);
    memcpy(&version, p + 8, 4);
    memcpy(&w32, p + 12, 4);
    memcpy(&nmax, p + 16, 4);
    memcpy(&ncls, p + 20, 4);
    memcpy(&sw, p + 24, 8);
    memcpy(&seed, p + 32, 8);
    if (magic != ORC_CKPT_MAGIC || version != 1 || w32 != (uint32_t)S || nmax != (uint32_t)c->n_max || ncls != 1 ||
        seed != c->seed || sw < 0)
        return -1;
    const char *pn = p + ORC_CKPT_HEADER, *pe = pn + S * 4, *pl = pe + S * 8, *pw = pl + S * 4, *px = pw + S * 4;
    const char *ps = px + S * (size_t)c->n_max * 3 * 8, *pa = ps + S * ORC_NSTAT * 8, *pc = pa + 4 * S * 8;
    for (size_t w = 0; w < S; ++w) {
        int32_t nn, lab, wo;
        memcpy(&nn, pn + 4 * w, 4);
        memcpy(&lab, pl + 4 * w, 4);
        if (nn < 0 || nn > c->n_max || lab < 0 || (size_t)lab >= S) return -1;
        memcpy(&wo, pw + 4 * (size_t)lab, 4);
        if ((size_t)wo != w) return -1;
    }
    memcpy(W->n, pn, S * 4);
    memcpy(W->e, pe, S * 8);
    memcpy(W->label, pl, S * 4);
    memcpy(W->wos, pw, S * 4);
    memcpy(W->xyz, px, S * (size_t)c->n_max * 3 * 8);
    memcpy(W->stats, ps, S * ORC_NSTAT * 8);
    memcpy(W->swap_att, pa, 4 * S * 8);
    memcpy(W->swap_acc, pc, 4 * S * 8);
    *sweep = sw;
    return 0;
}
