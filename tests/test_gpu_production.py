"""GPU parity at the sizes the product runs: the FP32 pair mode's long-run <N> on a
sub-grid of the 1024-replica system, energies after a production-length FP32 run,
the reweighting with 32 temperatures (the kernel instance the 32 x 32 grid uses),
the reweighting's error estimates, heat capacity and coverage, the FP32 sampler's
own network, and multi-step Adam.  Every expected value comes from the oracle
(oracle/ or oracle/mlp_oracle.py) on the same inputs."""
import math
import sys

import numpy as np
import pytest

import oracle
from oracle import mlp_oracle as M
from paper_1908_11118_amd import regc
from paper_1908_11118_amd import workloads as W
from tests.stats_util import batch_means, per_state_series

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build(force=False)
    torch.cuda.set_device(0)


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# (1) long-run <N> of the FP32 pair mode on the 1024-replica system's sub-grid
# ---------------------------------------------------------------------------
def _config2_subgrid(step=4, seed=1):
    """Every `step`-th temperature and chemical potential of the 32 x 32 grid of the
    192-atom, 12^3, N <= 200 system, run as its own REGC (8 x 8 = 64 replicas)."""
    w = W.config2()
    return w.replace(t=w.t[::step], mu=w.mu[::step], sample_every=1, seed=seed)


def test_fp32_config2_subgrid_mean_n_within_3se():
    """The oracle equilibrates the 64 replicas (2000 sweeps, FP64), then the oracle
    (seed 1) and the GPU in FP32 pair mode at the production launch shape (seed 2)
    both continue from that state for 3000 sweeps.  Per state, the difference of
    the mean N (first 10 % dropped) against the combined batch-means standard error
    (20 batches): at most one state beyond 3 SE (0.17 expected under the null), none
    beyond 4, and chi^2 per state of the z-scores <= 1.5."""
    w1 = _config2_subgrid(seed=1)
    S = w1.n_states
    burn, sweeps = 2000, 3000
    _say(f"[fp32 <N>] config2 sub-grid 8x8: oracle burn-in {burn} sweeps")
    ref = oracle.Chain(w1)
    ref.run(burn)
    n0, xyz0, lab0 = ref.n.copy(), ref.xyz.copy(), ref.label.copy()
    _say(f"[fp32 <N>] oracle {sweeps} sweeps")
    r = ref.run(sweeps)
    _say(f"[fp32 <N>] GPU {sweeps} sweeps")
    with regc.Regc(w1.replace(seed=2), precision=regc.FP32PAIR, sample_capacity=sweeps * S) as g:
        g.set_walkers(n0, xyz0, label=lab0)
        g.run(sweeps)
        smp = g.samples()
    cut = sweeps // 10
    n_ref = per_state_series(r, S)[0][cut:]
    n_gpu = per_state_series(smp, S)[0][cut:]
    z = np.zeros(S)
    for s in range(S):
        ma, sa = batch_means(n_gpu[:, s])
        mb, sb = batch_means(n_ref[:, s])
        se = math.sqrt(sa * sa + sb * sb)
        z[s] = (ma - mb) / se if se > 0 else (0.0 if ma == mb else np.inf)
    chi2 = float(np.mean(z * z))
    worst = int(np.argmax(np.abs(z)))
    msg = (f"|z| > 3 at {int(np.sum(np.abs(z) > 3))} states, max |z| {abs(z[worst]):.2f} (state {worst}), "
           f"chi2/state {chi2:.2f}")
    _say(f"[fp32 <N>] {msg}")
    assert np.sum(np.abs(z) > 3) <= 1, msg
    assert np.all(np.abs(z) <= 4), msg
    assert chi2 <= 1.5, msg


# ---------------------------------------------------------------------------
# (2) energies after a production-length FP32 run (running-energy resync)
# ---------------------------------------------------------------------------
def test_fp32_energies_after_ten_thousand_sweeps_config2():
    """1024 replicas, 10^4 + 50 sweeps in FP32 pair mode with the default resync (every
    100 sweeps): the running energies of the final configurations agree with the
    oracle's FP64 energies of the same configurations to 1e-5 relative."""
    w = W.config2()
    sweeps = 10_050
    _say(f"[fp32 resync] config2 1024 walkers, {sweeps} sweeps")
    with regc.Regc(w, precision=regc.FP32PAIR, sample_capacity=0, graph_intervals=10) as g:
        g.run(sweeps)
        wk = g.walkers()
    ch = oracle.Chain(w.replace(t=w.t[:1], mu=w.mu[:1]))
    rng = np.random.default_rng(3)
    idx = np.concatenate([np.argsort(wk["n"])[-32:], rng.choice(len(wk["n"]), 32, replace=False)])
    assert wk["n"].max() > 150
    worst = 0.0
    for k in idx:
        e_ref = ch.energy(wk["xyz"][k, : wk["n"][k]])
        rel = abs(wk["e"][k] - e_ref) / max(1.0, abs(e_ref))
        worst = max(worst, rel)
        assert rel <= 1e-5, (k, wk["n"][k], wk["e"][k], e_ref)
    _say(f"[fp32 resync] largest relative energy error {worst:.2e}")


# ---------------------------------------------------------------------------
# (3) reweighting with 32 temperatures against the naive oracle
# ---------------------------------------------------------------------------
def test_mbar_32_temperatures_matches_the_naive_oracle():
    """32 T x 2 mu states of the 32-atom system (the instance of the solve that a
    grid of 17..32 temperatures runs, as the 32 x 32 grid does), 6.4e4 samples of an
    oracle REGC run (the naive oracle's solve of them takes ~1700 plain iterations):
    free energies within 1e-7, <N>, <E> within 1e-7 relative, P(N) within 1e-8 and
    the phase map identical (wherever the top two probabilities differ by > 1e-9)."""
    w = W.config1().replace(t=W.linear_grid(0.5, 2.0, 32), mu=W.linear_grid(-5.0, -2.0, 2))
    S = w.n_states
    _say(f"[mbar 32 T] oracle run, {S} states")
    ch = oracle.Chain(w)
    ch.run(300)
    r = ch.run(1000)
    e, n, st = r["e"], r["n"], r["state"]
    keep = len(e)
    beta, lnz = oracle.state_arrays(w)
    omega = np.bincount(st, minlength=S)
    _say(f"[mbar 32 T] naive oracle solve over {keep} samples")
    f_ref, logd, ok, it, d = oracle.mbar_solve(beta, lnz, omega, e, n, tol=1e-10, max_iter=20000)
    assert ok, (it, d)
    mb = regc.Mbar(w.t, w.mu, w.n_max)
    mb.set_samples(e, n, st)
    f_gpu, conv, it_gpu, _ = mb.solve(tol=1e-10)
    assert conv
    assert np.abs(f_gpu - f_ref).max() <= 1e-7, np.abs(f_gpu - f_ref).max()
    tt = W.linear_grid(0.45, 2.1, 9)
    tm = W.linear_grid(-8.5, -1.5, 11)
    tb = np.repeat(1.0 / tt, len(tm))
    tz = np.array([oracle.state_lnz(T, u, w.lambda1) for T in tt for u in tm])
    ref = oracle.mbar_targets(tb, tz, e, n, logd, w.n_max)
    got = mb.targets(tt, tm)
    assert np.allclose(got["mean_n"], ref["mean_n"], rtol=1e-7, atol=1e-9)
    assert np.allclose(got["mean_e"], ref["mean_e"], rtol=1e-7, atol=1e-9)
    assert np.abs(got["p_n"] - ref["p_n"]).max() <= 1e-8
    top2 = np.sort(ref["p_n"], axis=1)[:, -2:]
    clear = (top2[:, 1] - top2[:, 0]) > 1e-9
    assert np.array_equal(got["phase"][clear], ref["phase"][clear])
    mb.close()
    _say(f"[mbar 32 T] oracle {it} iterations, GPU {it_gpu}")


# ---------------------------------------------------------------------------
# (4) errors, coverage and heat capacity of the reweighting
# ---------------------------------------------------------------------------
def test_reweight_errors_coverage_heat_capacity_match_the_oracle():
    """regc_reweight against the oracle's definitions on the same samples: the
    direct per-state means and their batch-means SE, the solution and averages, the
    heat capacity and coverage, and the bootstrap SEs of <N> and C (20 replicates of
    blocks of 10 records, the same Philox-keyed blocks on both sides)."""
    w = W.small_lj(n_t=2, n_mu=3, n_max=20, t=(0.9, 1.4), mu=(-6.0, -3.5))
    S = w.n_states
    ch = oracle.Chain(w)
    ch.run(200)
    r = ch.run(600)
    e, n, st = r["e"], r["n"], r["state"]
    beta, lnz = oracle.state_arrays(w)
    tt = np.array([0.9, 1.1, 1.4])
    tm = np.array([-6.0, -4.6, -3.5])
    n_sites = 16.0
    nb, nboot, blk, seed = 20, 20, 10, 5
    mb = regc.Mbar(w.t, w.mu, w.n_max)
    mb.set_samples(e, n, st)
    got = mb.reweight(tt, tm, tol=1e-12, n_batches=nb, n_boot=nboot, block_records=blk, seed=seed, n_sites=n_sites)
    assert got["converged"]
    # direct means at the sampled states
    m_ref, se_ref = oracle.batch_means(S, st, n, nb)
    assert np.allclose(got["mean_state_n"], m_ref, rtol=1e-14, atol=0)
    assert np.allclose(got["se_state_n"], se_ref, rtol=1e-12, atol=1e-15)
    # the solution and the averages at the targets
    f_ref, logd, ok, _, _ = oracle.mbar_solve(beta, lnz, np.bincount(st, minlength=S), e, n, tol=1e-12)
    assert ok and np.abs(got["f_states"] - f_ref).max() <= 1e-8
    tb = np.repeat(1.0 / tt, len(tm))
    tz = np.array([oracle.state_lnz(T, u, w.lambda1) for T in tt for u in tm])
    t_ref = oracle.mbar_targets(tb, tz, e, n, logd, w.n_max)
    hc_ref, cov_ref = oracle.heat_capacity_coverage(tb, t_ref["mean_n"], t_ref["mean_e"], t_ref["mean_e2"], n_sites)
    assert np.allclose(got["mean_n"], t_ref["mean_n"], rtol=1e-8)
    assert np.allclose(got["coverage"], cov_ref, rtol=1e-8)
    assert np.allclose(got["heat_cap"], hc_ref, rtol=1e-6, atol=1e-9)
    # bootstrap standard errors
    se_n, se_c, rn, rc, ok = oracle.mbar_bootstrap(beta, lnz, e, n, st, S, blk, nboot, seed, f_ref, tb, tz, w.n_max,
                                                   tol=1e-12)
    assert ok
    assert np.all(se_n > 0) and np.all(se_c > 0)
    assert np.allclose(got["se_n"], se_n, rtol=1e-5, atol=1e-10), (got["se_n"], se_n)
    assert np.allclose(got["se_coverage"], se_n / n_sites, rtol=1e-5, atol=1e-10)
    assert np.allclose(got["se_heat_cap"], se_c, rtol=1e-4, atol=1e-8), (got["se_heat_cap"], se_c)
    # the handle still holds the full-data solution
    again = mb.targets(tt, tm)
    assert np.allclose(again["mean_n"], t_ref["mean_n"], rtol=1e-8)
    mb.close()


def test_batch_means_entry_matches_the_oracle():
    """regc_batch_means (host and device inputs) against the oracle's batch means on
    an uneven per-state sample count, a state below the batch count, and rejection of
    an out-of-range state."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(21)
    S, ns = 37, 250_000
    st = rng.integers(0, S - 1, ns).astype(np.int32)          # state S-1 gets a handful only
    st[:7] = S - 1
    n = rng.poisson(3.0 + st % 11, ns).astype(np.int32)
    m_ref, se_ref = oracle.batch_means(S, st, n, 20)
    m, se = regc.batch_means(st, n, S, 20)
    assert np.array_equal(np.isnan(m), np.isnan(m_ref)) and np.isnan(m[S - 1])
    ok = ~np.isnan(m_ref)
    assert np.allclose(m[ok], m_ref[ok], rtol=1e-14, atol=0)
    assert np.allclose(se[ok], se_ref[ok], rtol=1e-12, atol=1e-15)
    md, sed = regc.batch_means(torch.from_numpy(st).cuda(), torch.from_numpy(n).cuda(), S, 20)
    assert np.array_equal(md[ok], m[ok]) and np.array_equal(sed[ok], se[ok])
    bad = st.copy()
    bad[100] = S
    with pytest.raises(regc.RegcError) as ei:
        regc.batch_means(bad, n, S, 20)
    assert ei.value.code == regc.EINVAL


def test_running_series_of_the_time_to_accuracy_matches_the_oracle():
    """The time-to-accuracy runs' sample series (records added chunk by chunk, statistics
    from regc_batch_means) against the oracle's batch means over all samples, whatever
    the chunking; infinite SE before 20 samples per state."""
    from paper_1908_11118_amd.proposal import _Series
    rng = np.random.default_rng(0)
    S, recs = 8, 1013
    state = np.array([rng.permutation(S) for _ in range(recs)]).ravel().astype(np.int32)
    n = rng.integers(0, 50, recs * S).astype(np.int32)
    m_ref, se_ref = oracle.batch_means(S, state, n, 20)
    for chunk in (1, 37, 100, recs):
        ser = _Series(S)
        for k in range(0, recs, chunk):
            ser.add(state[k * S:(k + chunk) * S], n[k * S:(k + chunk) * S])
        m, se = ser.mean_se()
        assert np.allclose(m, m_ref, rtol=0, atol=1e-12)
        assert np.allclose(se, se_ref, rtol=1e-12, atol=1e-12)
    few = _Series(3)
    few.add(np.tile(np.arange(3, dtype=np.int32), 10), rng.integers(0, 9, 30).astype(np.int32))
    m, se = few.mean_se()
    assert np.all(np.isinf(se)) and np.all(np.isnan(m))


def test_reweight_rejects_partial_records():
    w = W.small_lj(n_t=2, n_mu=2, n_max=10)
    mb = regc.Mbar(w.t, w.mu, w.n_max)
    rng = np.random.default_rng(0)
    mb.set_samples(rng.normal(-5, 1, 10), rng.integers(0, 10, 10), np.arange(10) % 4)
    with pytest.raises(regc.RegcError) as ei:
        mb.reweight(w.t, w.mu, n_boot=10)          # 10 samples are not whole records of 4
    assert ei.value.code == regc.EINVAL
    mb.close()


# ---------------------------------------------------------------------------
# (5) the FP32 sampler's own network, element by element
# ---------------------------------------------------------------------------
def _net_params(seed):
    p = W.mlp_init(seed, out_scale=3.0)
    rng = np.random.default_rng(seed + 7)
    for k in ("b1", "b2", "b3", "b4"):
        p[k] = rng.normal(0, 0.3, p[k].shape).astype(np.float32)
    return p


def _configurations(w, rng):
    confs, ns, skips = [], [], []
    for n in (0, 1, 3, 7, 12, 20, 28, 35, 40, 40):
        x = W.random_configuration(rng, w, n, min_dist=0.7) if n else np.zeros((0, 3))
        x = x.astype(np.float32).astype(np.float64)           # positions the FP32 sampler holds exactly
        confs.append(x)
        ns.append(n)
        skips.append(int(rng.integers(0, n)) if n and rng.random() < 0.6 else -1)
    return confs, np.array(ns, np.int32), np.array(skips, np.int32)


def test_fp32_sampler_network_matches_the_bf16_oracle():
    """The FP32 build's network (MFMA layers on the sampler's packed tiles, FP32
    log-normaliser) on configurations with and without a left-out particle: logits
    within 1e-3 of the largest against the oracle's bfloat16-emulating forward, the
    log-normaliser within 1e-3, and the probabilities the acceptance uses normalised
    to 1e-12 (they are the voxel draw's own weights)."""
    w = W.config1()
    p = _net_params(3)
    rng = np.random.default_rng(8)
    confs, ns, skips = _configurations(w, rng)
    net = regc.Mlp(W.mlp_pack(p))
    with regc.Regc(w, precision=regc.FP32PAIR, sample_capacity=0) as g:
        g.set_proposal(net, 0.9)
        lg, lse, lnp = g.proposal_eval(ns, confs, skips)
    net.close()
    vox = np.zeros((len(ns), w.n_max), np.uint16)
    for k, x in enumerate(confs):
        if len(x):
            vox[k, : len(x)] = M.voxel_of(x, w.lx, w.ly, w.zlo, w.zhi)
    ref = M.forward(p, vox, ns, skips, "bf16")["logits"].astype(np.float64)
    scale = np.abs(ref).max()
    err = np.abs(lg - ref).max() / scale
    assert err <= 1e-3, err
    ref_lse = ref.max(1) + np.log(np.exp(ref - ref.max(1, keepdims=True)).sum(1))
    assert np.abs(lse - ref_lse).max() <= 1e-3 * scale
    assert np.abs(np.exp(lnp).sum(1) - 1.0).max() <= 1e-12
    big = lnp > -20
    assert np.abs(lnp[big] - (ref - ref_lse[:, None])[big]).max() <= 2e-3 * scale


def test_fp64_sampler_network_is_the_oracles_bit_for_bit():
    w = W.config1()
    p = _net_params(4)
    flat = W.mlp_pack(p)
    rng = np.random.default_rng(9)
    confs, ns, skips = _configurations(w, rng)
    net = regc.Mlp(flat)
    with regc.Regc(w, precision=regc.FP64, sample_capacity=0) as g:
        g.set_proposal(net, 0.9)
        lg, lse, lnp = g.proposal_eval(ns, confs, skips)
    net.close()
    ch = oracle.Chain(w, net=flat, alpha=0.9)
    for k, x in enumerate(confs):
        ref, ref_lse = ch.net_logits(x, int(skips[k]))
        assert np.array_equal(lg[k], ref), k
        assert abs(lse[k] - ref_lse) <= 1e-12 * max(1.0, abs(ref_lse))


# ---------------------------------------------------------------------------
# (6) Adam over several steps against the oracle's Adam on the same gradients
# ---------------------------------------------------------------------------
def test_adam_three_steps_match_the_oracle():
    """Three Adam steps on three different batches: the GPU's parameters (FP32) equal
    the oracle's Adam (FP64) applied to the same starting parameters and the
    gradients the GPU applied, to 1e-6 of the parameter scale; the first gradient
    matches the oracle's bfloat16 gradient within 1e-3 of its largest entry."""
    rng = np.random.default_rng(11)
    p0 = _net_params(5)
    for k in p0:
        p0[k] = (p0[k] * 0.3).astype(np.float32)
    net = regc.Mlp(W.mlp_pack(p0))
    ref = {k: v.astype(np.float64) for k, v in p0.items()}
    state = {}
    lr = 2e-3
    for step in range(3):
        B, nmax = 64, 40
        n = rng.integers(1, nmax + 1, B).astype(np.int32)
        vox = rng.integers(0, 4096, (B, nmax)).astype(np.uint16)
        excl = np.array([rng.integers(0, k) for k in n], np.int32)
        target = np.array([vox[b, excl[b]] for b in range(B)], np.int32)
        if step == 0:
            _, g_ref = M.loss_and_grads(p0, vox, n, excl, target, "bf16")
        loss, g = net.step(vox, n, excl, target, lr=lr)
        gd = {k: v.astype(np.float64) for k, v in W.mlp_unpack(g).items()}
        if step == 0:
            for k in W.MLP_ORDER:
                sc = np.abs(g_ref[k]).max()
                assert np.abs(gd[k] - g_ref[k]).max() <= 1e-3 * sc, k
        M.adam(ref, gd, state, lr=lr)
    got = W.mlp_unpack(net.params())
    net.close()
    for k in W.MLP_ORDER:
        scale = max(1.0, np.abs(ref[k]).max())
        err = np.abs(got[k].astype(np.float64) - ref[k]).max()
        assert err <= 1e-6 * scale, (k, err)
        moved = np.abs(ref[k] - p0[k].astype(np.float64)).max()
        assert moved > 0.5 * lr, (k, moved)       # three steps really moved the parameters
