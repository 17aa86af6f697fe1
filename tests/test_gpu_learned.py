"""GPU parity of sampling with the learned insertion proposal, through the C ABI.

FP64 build: the sampler's network arithmetic reproduces the oracle's bit for bit,
so trajectories (accept bits, N, labels, statistics) must be identical to the
oracle's learned chain and energies agree to 1e-10.  FP32 build (MFMA network):
the stationary law is checked -- the ideal-gas Poisson mean under a random network
and under a fixed proposal peaked on 16 voxels (with uniform positions, which tests
the inverse-CDF voxel draw), and the LJ mean N of the plain FP64 oracle, within 3
standard errors over the states (tests/stats_util.assert_within_3se)."""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_1908_11118_amd import regc
from paper_1908_11118_amd import workloads as W
from tests.stats_util import assert_within_3se, batch_means, per_state_series, truncated_poisson

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


def _net(seed, out_scale=3.0):
    p = W.mlp_init(seed, out_scale=out_scale)
    rng = np.random.default_rng(seed + 7)
    for k in ("b1", "b2", "b3", "b4"):
        p[k] = rng.normal(0, 0.3, p[k].shape).astype(np.float32)
    return W.mlp_pack(p)


def _first_divergence(bits_a, bits_b, n_a, n_b):
    d = np.argwhere(bits_a != bits_b)
    if len(d):
        s, w, word = d[0]
        x = int(bits_a[s, w, word] ^ bits_b[s, w, word])
        return f"sweep {s} walker {w} trial {32 * word + (x & -x).bit_length() - 1}"
    d = np.argwhere(n_a != n_b)
    if len(d):
        return f"N differs at sweep {d[0][0]} walker {d[0][1]}"
    return None


def _learned_trajectory(w, sweeps, params, alpha, **kw):
    _say(f"[learned fp64] {w.name} S={w.n_states} sweeps={sweeps} alpha={alpha} {kw}")
    ref = oracle.Chain(w, net=params, alpha=alpha)
    r = ref.run(sweeps, trace=True, margins=True)
    net = regc.Mlp(params)
    with regc.Regc(w, precision=regc.FP64, trace_capacity=sweeps, sample_capacity=0, **kw) as g:
        g.set_proposal(net, alpha)
        g.run(sweeps)
        bits, nps = g.trace(sweeps)
        wk = g.walkers()
        st = g.stats()
        ps = g.proposal_stats()
    net.close()
    where = _first_divergence(bits, r["bits"], nps, r["trace_n"])
    assert where is None, f"trajectory diverges: {where} (oracle margin min {np.min(r['margin']):.3g})"
    assert np.array_equal(wk["n"], ref.n)
    assert np.array_equal(wk["label"], ref.label)
    assert np.allclose(wk["e"], ref.e, rtol=1e-10, atol=1e-9)
    for k in range(ref.S):
        assert np.allclose(wk["xyz"][k, : ref.n[k]], ref.xyz[k, : ref.n[k]], rtol=0, atol=1e-12)
    assert np.array_equal(st["stats"], ref.stats)
    assert np.array_equal(st["swap_att"], ref.swap_att)
    assert np.array_equal(st["swap_acc"], ref.swap_acc)
    return ref, ps


def test_learned_fp64_trajectories_config1():
    """64 replicas of the 32-atom slab system, a random network, alpha = 0.5,
    200 sweeps with exchanges: identical decisions, the network used throughout."""
    ref, ps = _learned_trajectory(W.config1(), 200, _net(1), 0.5)
    st = ref.stats.sum(0)
    assert ps["drawn"] > 1000 and ps["drawn_accepted"] > 0
    assert ps["passes"] > st[oracle.STAT_NAMES.index("del_att")] // 2
    assert ps["cached"] > 0


@pytest.mark.parametrize("alpha,graph", [(1.0, 0), (0.05, 2), (0.7, 0)])
def test_learned_fp64_small_systems(alpha, graph):
    w = W.small_lj(n_t=2, n_mu=3, n_max=16, n_sweeps=200, mu=(-4.0, -2.0))
    _learned_trajectory(w, 200, _net(2), alpha, graph_intervals=graph)


def test_learned_fp64_dense_walkers():
    """N above a wavefront's width and a binned 8x8x3 slab: every wave owns gas
    candidates and the occupied-voxel list spans several threads' ranges."""
    w = W.config2(40).replace(t=np.array([0.9, 1.6]), mu=np.array([-3.0, -2.0]), n_max=140, sample_every=0)
    ref, _ = _learned_trajectory(w, 40, _net(3, out_scale=1.5), 0.8)
    assert ref.n.max() > 80


def test_learned_fp64_ideal_gas_and_edges():
    _learned_trajectory(W.ideal_gas(n_t=2, n_mu=2, n_max=30), 200, _net(4), 0.9)
    # N capped at 1, one trial per sweep
    _learned_trajectory(W.small_lj(n_t=1, n_mu=2, n_max=1).replace(swap_every=0), 300, _net(5), 0.9)
    _learned_trajectory(W.small_lj(n_t=2, n_mu=2, n_max=8).replace(trials_per_sweep=1), 300, _net(5), 0.9)


def test_alpha_zero_and_errors():
    w = W.small_lj(n_t=2, n_mu=2, n_max=12)
    net = regc.Mlp(_net(6))
    ref = oracle.Chain(w)
    r = ref.run(100, trace=True)
    with regc.Regc(w, precision=regc.FP64, trace_capacity=100, sample_capacity=0) as g:
        g.set_proposal(net, 0.7)
        g.set_proposal(net, 0.0)            # back to the plain method
        g.run(100)
        bits, nps = g.trace(100)
        with pytest.raises(regc.RegcError):
            g.set_proposal(net, 1.5)
    assert _first_divergence(bits, r["bits"], nps, r["trace_n"]) is None
    with regc.Regc([w, w.replace(seed=3)], precision=regc.FP64, sample_capacity=0) as g:
        with pytest.raises(regc.RegcError):
            g.set_proposal(net, 0.5, cls=2)          # no such class
        with pytest.raises(regc.RegcError):
            g.set_proposal(net, -0.1, cls=0)
    with regc.Regc(W.paper_schedule(w), precision=regc.FP64, sample_capacity=0) as g:
        with pytest.raises(regc.RegcError):
            g.set_proposal(net, 0.5)                 # the paper's step keeps uniform insertion
    net.close()


def _batch_classes():
    """Three slab classes of different box, n_max and grid (swaps within a class)."""
    c3 = W.config3_classes()
    out = [c3[1].replace(t=W.linear_grid(0.6, 1.8, 3), mu=W.linear_grid(-5.0, -2.5, 4), n_max=70),
           W.small_lj(n_t=2, n_mu=3, n_max=30, mu=(-4.0, -2.0)),
           c3[0].replace(t=W.linear_grid(0.7, 1.5, 4), mu=W.linear_grid(-6.0, -3.0, 2), n_max=50)]
    return [w.replace(sample_every=3, swap_every=10) for w in out]


@pytest.mark.parametrize("graph", [0, 2])
def test_learned_fp64_uneven_batch_one_network_per_class(graph):
    """A batch of three slab classes in the same launches, each class with its own
    network over its own box (the last class without one, inserting uniformly):
    every class's trajectories equal a lone oracle learned chain with the batch's
    walker offsets; with graph replay of whole exchange intervals too."""
    classes = _batch_classes()
    setup = [(_net(11), 0.6), (None, 0.0), (_net(12, out_scale=2.0), 0.9)]
    sweeps = 45
    _say(f"[learned batch] {len(classes)} classes, graph={graph}")
    nets = [regc.Mlp(p) if p is not None else None for p, _ in setup]
    with regc.Regc(classes, precision=regc.FP64, trace_capacity=sweeps, graph_intervals=graph,
                   sample_capacity=0) as g:
        for c, (net, (_, alpha)) in enumerate(zip(nets, setup)):
            g.set_proposal(net, alpha, cls=c)
        g.run(20)
        g.run(sweeps - 20)
        bits, nps = g.trace(sweeps)
        wk = g.walkers()
        st = g.stats()
        ps = g.proposal_stats()
        offs, cnts = g.offsets, g.counts
    for net in nets:
        if net is not None:
            net.close()
    assert ps["drawn"] > 0 and ps["passes"] > 0
    for c, w in enumerate(classes):
        params, alpha = setup[c]
        ref = oracle.Chain(w, walker_offset=offs[c], class_id=c, net=params, alpha=alpha)
        r = ref.run(sweeps, trace=True)
        sl = slice(offs[c], offs[c] + cnts[c])
        words = r["bits"].shape[2]
        where = _first_divergence(bits[:, sl, :words], r["bits"], nps[:, sl], r["trace_n"])
        assert where is None, f"class {c}: {where}"
        assert np.array_equal(wk["n"][sl], ref.n) and np.array_equal(wk["label"][sl], ref.label)
        assert np.allclose(wk["e"][sl], ref.e, rtol=1e-10, atol=1e-9)
        assert np.array_equal(st["stats"][sl], ref.stats)
        assert np.array_equal(st["swap_acc"][:, sl], ref.swap_acc)


def test_learned_fp32_ideal_gas_poisson():
    """MFMA network, random weights, alpha = 0.9: the stationary law is still the
    truncated Poisson of mean zV."""
    w = W.ideal_gas(n_max=24).replace(t=W.linear_grid(0.9, 1.3, 3), mu=W.linear_grid(-4.6, -3.8, 3),
                                      swap_every=10, sample_every=1)
    sweeps = 12000
    _say(f"[learned fp32 poisson] S={w.n_states} sweeps={sweeps}")
    net = regc.Mlp(_net(7))
    with regc.Regc(w, precision=regc.FP32PAIR, sample_capacity=sweeps * w.n_states) as g:
        g.set_proposal(net, 0.9)
        g.run(1000)
        g.clear_samples()
        g.run(sweeps)
        smp = g.samples()
        ps = g.proposal_stats()
    net.close()
    n_ser, _ = per_state_series(smp, w.n_states)
    z = []
    for s in range(w.n_states):
        T, mu = w.t[s // len(w.mu)], w.mu[s % len(w.mu)]
        zv = math.exp(mu / T) * T ** 1.5 * w.volume
        p = truncated_poisson(zv, w.n_max)
        mean_ref = float((np.arange(w.n_max + 1) * p).sum())
        m, se = batch_means(n_ser[:, s])
        z.append((m - mean_ref) / se)
    assert_within_3se(z, "ideal gas, random network")
    assert ps["drawn"] > 0 and ps["drawn_accepted"] > 0


def test_learned_fp32_draw_of_a_peaked_proposal():
    """W4 = 0 and an output bias of 6 on 16 voxels: q is fixed, 61 % of it on 1/256 of
    the box, and alpha = 1, so every insertion comes from the FP32 build's voxel draw.
    The chain must still sample the ideal gas -- truncated-Poisson <N> per state and
    uniform positions (the 16 peaked voxels hold 16/4096 of the particles) -- which
    fails if the draw's law is not the q the acceptance divides by."""
    import torch
    w = W.ideal_gas(n_max=24).replace(t=W.linear_grid(0.9, 1.3, 4), mu=W.linear_grid(-4.6, -3.8, 4),
                                      swap_every=10, sample_every=1)
    p = W.mlp_init(3)
    p["W4"][:] = 0.0
    hot = np.random.default_rng(5).choice(4096, 16, replace=False)
    p["b4"][hot] = 6.0
    net = regc.Mlp(W.mlp_pack(p))
    sweeps, every = 8000, 20
    nw = w.n_states
    _say(f"[learned fp32 peaked] S={nw} sweeps={sweeps}")
    vox = torch.zeros((nw, w.n_max), dtype=torch.int16, device="cuda")
    nd = torch.zeros(nw, dtype=torch.int32, device="cuda")
    in_hot = total = 0
    with regc.Regc(w, precision=regc.FP32PAIR, sample_capacity=sweeps * nw) as g:
        g.set_proposal(net, 1.0)
        g.run(1000)
        g.clear_samples()
        for _ in range(sweeps // every):
            g.run(every)
            g.capture_voxels(vox.data_ptr(), nd.data_ptr())
            g.sync()
            torch.cuda.synchronize()
            v = vox.cpu().numpy().astype(np.int64) & 0xFFFF
            keep = np.arange(w.n_max)[None, :] < nd.cpu().numpy()[:, None]
            in_hot += int(np.isin(v[keep], hot).sum())
            total += int(keep.sum())
        smp = g.samples()
        ps = g.proposal_stats()
    net.close()
    n_ser, _ = per_state_series(smp, nw)
    z = []
    for s in range(nw):
        T, mu = w.t[s // len(w.mu)], w.mu[s % len(w.mu)]
        zv = math.exp(mu / T) * T ** 1.5 * w.volume
        pr = truncated_poisson(zv, w.n_max)
        mean_ref = float((np.arange(w.n_max + 1) * pr).sum())
        m, se = batch_means(n_ser[:, s])
        z.append((m - mean_ref) / se)
    assert_within_3se(z, "ideal gas, peaked proposal")
    expected = 16.0 / 4096.0
    assert total > 20000 and abs(in_hot / total - expected) < 0.3 * expected, (in_hot, total, expected)
    assert ps["drawn"] > 0 and ps["drawn_accepted"] > 0


def test_learned_fp32_lj_mean_n_matches_the_plain_oracle():
    w = W.small_lj(n_t=2, n_mu=2, n_max=16, mu=(-4.5, -3.0)).replace(sample_every=1)
    sweeps = 20000
    _say(f"[learned fp32 lj] sweeps={sweeps}")
    ref = oracle.Chain(w)
    ref.run(1000)
    r = ref.run(sweeps)
    net = regc.Mlp(_net(8, out_scale=2.0))
    with regc.Regc(w, precision=regc.FP32PAIR, sample_capacity=sweeps * w.n_states) as g:
        g.set_proposal(net, 0.7)
        g.run(1000)
        g.clear_samples()
        g.run(sweeps)
        smp = g.samples()
    net.close()
    na, _ = per_state_series(r, w.n_states)
    nb, _ = per_state_series(smp, w.n_states)
    z = []
    for s in range(w.n_states):
        ma, sa = batch_means(na[:, s])
        mb, sb = batch_means(nb[:, s])
        z.append((ma - mb) / math.hypot(sa, sb))
    assert_within_3se(z, "LJ, learned FP32 against the plain oracle")


def test_learned_fp32_batch_one_network_per_class_mean_n():
    """The full stack at a small size: two slab classes of different box in one
    batch, each with its own MFMA network (random weights) in the sweep, FP32 pairs:
    every state's mean N agrees with the plain FP64 oracle run of that class within
    3 standard errors (over the states of both classes)."""
    classes = [W.small_lj(n_t=2, n_mu=2, n_max=14, mu=(-4.5, -3.0)).replace(sample_every=1),
               W.small_lj(n_t=2, n_mu=2, n_max=18, box=7.5, height=5.0, mu=(-4.0, -3.0)).replace(sample_every=1)]
    sweeps = 16000
    _say(f"[learned fp32 batch] {len(classes)} classes sweeps={sweeps}")
    nets = [regc.Mlp(_net(21, out_scale=2.0)), regc.Mlp(_net(22, out_scale=2.0))]
    with regc.Regc(classes, precision=regc.FP32PAIR, sample_capacity=sweeps * sum(w.n_states for w in classes)) as g:
        g.set_proposal(nets[0], 0.7, cls=0)
        g.set_proposal(nets[1], 0.9, cls=1)
        g.run(1000)
        g.clear_samples()
        g.run(sweeps)
        smp = g.samples()
        ps = g.proposal_stats()
        offs, cnts = g.offsets, g.counts
    for net in nets:
        net.close()
    assert ps["drawn"] > 0 and ps["drawn_accepted"] > 0
    W_all = sum(cnts)
    z = []
    for c, w in enumerate(classes):
        ref = oracle.Chain(w, walker_offset=offs[c], class_id=c)
        ref.run(1000)
        r = ref.run(sweeps)
        sl = slice(offs[c], offs[c] + cnts[c])
        mine = {k: smp[k].reshape(-1, W_all)[:, sl].ravel() for k in ("n", "e", "state")}
        na, _ = per_state_series(r, w.n_states)
        nb, _ = per_state_series(mine, w.n_states)
        for s in range(w.n_states):
            ma, sa = batch_means(na[:, s])
            mb, sb = batch_means(nb[:, s])
            z.append((ma - mb) / math.hypot(sa, sb))
    assert_within_3se(z, "batch of two classes, one network each")
