"""Pins of the oracle's learned insertion proposal (an extension of the method):
the plain chain at alpha = 0, the ideal-gas Poisson law and an LJ long-run mean
under a random network, the network against the independent numpy network
oracle, Gumbel-max frequencies against the softmax, and the voxel map.  CPU only."""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp_oracle as M
from paper_1908_11118_amd import workloads as W
from tests.stats_util import batch_means, per_state_series, truncated_poisson


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def _net(seed, out_scale=3.0):
    p = W.mlp_init(seed, out_scale=out_scale)
    rng = np.random.default_rng(seed + 7)
    for k in ("b1", "b2", "b3", "b4"):
        p[k] = rng.normal(0, 0.3, p[k].shape).astype(np.float32)
    return p


def test_alpha_zero_is_the_plain_chain():
    w = W.small_lj(n_sweeps=60)
    plain = oracle.Chain(w)
    a = plain.run(60, trace=True)
    learned = oracle.Chain(w, net=W.mlp_pack(_net(1)), alpha=0.0)
    b = learned.run(60, trace=True)
    assert np.array_equal(a["bits"], b["bits"])
    assert np.array_equal(a["trace_n"], b["trace_n"])
    assert np.array_equal(plain.e, learned.e)
    assert np.array_equal(plain.xyz, learned.xyz)


def test_voxel_map():
    w = W.config1()
    ch = oracle.Chain(w)
    assert ch.voxel_of([0.0, 0.0, w.zlo]) == 0
    assert ch.voxel_of([w.lx - 1e-12, w.ly - 1e-12, w.zhi]) == 4095
    # the centre of cell (ix, iy, iz)
    rng = np.random.default_rng(3)
    for _ in range(50):
        ix, iy, iz = rng.integers(0, 16, 3)
        p = [(ix + 0.5) * w.lx / 16, (iy + 0.5) * w.ly / 16, w.zlo + (iz + 0.5) * (w.zhi - w.zlo) / 16]
        assert ch.voxel_of(p) == (iz * 16 + iy) * 16 + ix
        assert ch.voxel_of(p) == int(M.voxel_of(p, w.lx, w.ly, w.zlo, w.zhi)[0])


def test_network_matches_numpy_oracle():
    w = W.config1()
    p = _net(2)
    ch = oracle.Chain(w, net=W.mlp_pack(p), alpha=0.5)
    rng = np.random.default_rng(4)
    for n, skip in ((0, -1), (1, 0), (17, -1), (40, 13), (40, 39)):
        xyz = np.column_stack([rng.uniform(0, w.lx, n), rng.uniform(0, w.ly, n), rng.uniform(w.zlo, w.zhi, n)])
        if n >= 6:
            xyz[5] = xyz[2] + 1e-3           # two particles in one voxel
        got, lse = ch.net_logits(xyz, skip)
        vox = M.voxel_of(xyz, w.lx, w.ly, w.zlo, w.zhi).astype(np.int64).reshape(1, -1)
        if n == 0:
            vox = np.zeros((1, 1), np.int64)
        ref = M.forward(p, vox, np.array([n]), np.array([skip]), "bf16")["logits"][0]
        scale = np.abs(ref).max()
        assert np.abs(got - ref).max() <= 2e-5 * scale, (n, np.abs(got - ref).max() / scale)
        ref64 = M.forward({k: v.astype(np.float64) for k, v in p.items()}, vox, np.array([n]),
                          np.array([skip]), "fp64")["logits"][0]
        assert np.abs(got - ref64).max() <= 5e-2 * scale
        lp = M.log_softmax(got.astype(np.float64)[None])[0]
        assert abs((float(got[0]) - lse) - lp[0]) < 1e-9


def test_gumbel_max_frequencies_follow_the_softmax():
    w = W.config1()
    ch = oracle.Chain(w, net=W.mlp_pack(_net(3)), alpha=1.0)
    logits = np.zeros(4096, np.float32)
    top = [7, 100, 2048, 4095]
    logits[top] = [6.0, 5.5, 5.0, 4.0]
    prob = np.exp(logits.astype(np.float64))
    prob /= prob.sum()
    n = 6000
    draws = np.array([ch.gumbel_argmax(logits, t % 41, t // 41, 5)[0] for t in range(n)])
    for v in top:
        f = (draws == v).mean()
        sd = math.sqrt(prob[v] * (1 - prob[v]) / n)
        assert abs(f - prob[v]) < 4 * sd, (v, f, prob[v])
    rest = ~np.isin(draws, top)
    pr = 1 - prob[top].sum()
    assert abs(rest.mean() - pr) < 4 * math.sqrt(pr * (1 - pr) / n)
    # the counters, not the logits, carry the randomness: equal logits give a uniform draw
    flat = np.zeros(4096, np.float32)
    d2 = np.array([ch.gumbel_argmax(flat, t, 0, 0)[0] for t in range(4000)])
    hist = np.bincount(d2 // 256, minlength=16)
    chi2 = ((hist - 250.0) ** 2 / 250.0).sum()
    assert chi2 < 45.0                  # 15 dof, p ~ 1e-4


@pytest.mark.parametrize("swap_every", [0, 10])
def test_ideal_gas_poisson_with_a_random_network(swap_every):
    w = W.ideal_gas(n_max=16).replace(t=np.array([1.0, 1.2]), mu=np.array([-4.5, -4.0]),
                                      swap_every=swap_every, n_sweeps=3000)
    ch = oracle.Chain(w, net=W.mlp_pack(_net(5)), alpha=0.9)
    ch.run(200)
    out = ch.run(w.n_sweeps)
    n_ser, _ = per_state_series(out, ch.S)
    for s in range(ch.S):
        T, mu = w.t[s // 2], w.mu[s % 2]
        zv = math.exp(mu / T) * T ** 1.5 * w.volume
        p = truncated_poisson(zv, w.n_max)
        mean_ref = float((np.arange(w.n_max + 1) * p).sum())
        m, se = batch_means(n_ser[:, s])
        assert abs(m - mean_ref) < 4 * se + 1e-9, (s, m, mean_ref, se)
    st = ch.stats.sum(0)
    assert st[oracle.STAT_NAMES.index("ins_acc")] > 0.2 * st[oracle.STAT_NAMES.index("ins_att")]


def test_lj_mean_n_agrees_with_the_plain_chain():
    w = W.small_lj(n_sweeps=3000, mu=(-5.0, -3.5))
    plain = oracle.Chain(w)
    plain.run(300)
    a = plain.run(w.n_sweeps)
    learned = oracle.Chain(w, net=W.mlp_pack(_net(6, out_scale=2.0)), alpha=0.7)
    learned.run(300)
    b = learned.run(w.n_sweeps)
    na, _ = per_state_series(a, plain.S)
    nb, _ = per_state_series(b, learned.S)
    for s in range(plain.S):
        ma, sa = batch_means(na[:, s])
        mb, sb = batch_means(nb[:, s])
        assert abs(ma - mb) < 4 * math.hypot(sa, sb) + 1e-9, (s, ma, mb, sa, sb)
