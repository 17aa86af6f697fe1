"""Pins of the oracle's molecular-dynamics canonical part of the REGC step
(Sec. II.A; velocity Verlet with the stochastic velocity-rescaling thermostat):
forces against finite differences of the energy, energy conservation without the
thermostat, the ideal-gas Poisson law with equipartition and uniform density under
the thermostat, and the LJ mean N of the Monte Carlo schedule.  CPU only."""
import math

import numpy as np
import pytest

import oracle
from paper_1908_11118_amd import workloads as W
from tests.stats_util import batch_means, per_state_series, truncated_poisson


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def test_forces_are_minus_the_energy_gradient():
    w = W.config1()
    ch = oracle.Chain(w)
    rng = np.random.default_rng(2)
    xyz = W.random_configuration(rng, w, 25, min_dist=0.95)
    e, f = ch.md_forces(xyz)
    assert abs(e - ch.energy(xyz)) < 1e-10 * max(1.0, abs(e))
    h = 1e-6
    for i in range(0, 25, 3):
        for k in range(3):
            xp, xm = xyz.copy(), xyz.copy()
            xp[i, k] += h
            xm[i, k] -= h
            fd = -(ch.energy(xp) - ch.energy(xm)) / (2 * h)
            assert abs(fd - f[i, k]) < 1e-5 * max(1.0, abs(f[i, k])), (i, k, fd, f[i, k])


def test_energy_is_conserved_without_thermostat():
    w = W.small_lj(n_t=1, n_mu=1, n_max=20, mu=(-3.0, -3.0)).replace(swap_every=0, seed=3)
    mc = oracle.Chain(w)
    mc.run(500)                                       # an equilibrated configuration
    md = oracle.Chain(W.paper_schedule_md(w, x0=0.0, md_steps=1, md_dt=0.002, md_tau=0.0, sample_every=0))
    md.set_walkers(mc.n, mc.xyz)
    md.run(1)
    e0 = md.e[0] + 0.5 * (md.vel[0, : md.n[0]] ** 2).sum()
    k0 = 0.5 * (md.vel[0, : md.n[0]] ** 2).sum()
    for _ in range(5):
        md.run(100)
    e1 = md.e[0] + 0.5 * (md.vel[0, : md.n[0]] ** 2).sum()
    assert md.n[0] == mc.n[0] and md.n[0] > 5
    assert abs(e1 - e0) < 2e-3 * k0, (e0, e1, k0)


def test_ideal_gas_with_thermostat():
    w = W.paper_schedule_md(W.ideal_gas(n_max=25).replace(t=np.array([1.0, 1.5]), mu=np.array([-4.3, -3.7])),
                            x0=0.9, md_steps=5, md_dt=0.01, md_tau=0.05, sample_every=1)
    ch = oracle.Chain(w)
    ch.run(500)
    kin, eq, zs = [], [], []
    out_n, out_s = [], []
    for _ in range(60):
        r = ch.run(100)
        out_n.append(r["n"])
        out_s.append(r["state"])
        T = 1.0 / oracle.state_arrays(w)[0][ch.label]
        kin.append(sum(0.5 * (ch.vel[k, : ch.n[k]] ** 2).sum() for k in range(ch.S)))
        eq.append(sum(1.5 * ch.n[k] * T[k] for k in range(ch.S)))
        zs.extend(ch.xyz[k, j, 2] for k in range(ch.S) for j in range(ch.n[k]))
    assert abs(np.sum(kin) / np.sum(eq) - 1.0) < 0.05
    # uniform in [z_lo, z_hi] between the reflecting walls (snapshots 100 steps apart,
    # counted as half independent)
    sd = (w.zhi - w.zlo) / math.sqrt(12.0)
    assert abs(np.mean(zs) - 0.5 * (w.zlo + w.zhi)) < 4 * sd * math.sqrt(2.0 / len(zs))
    n_ser, _ = per_state_series({"n": np.concatenate(out_n), "state": np.concatenate(out_s),
                                 "e": np.zeros(sum(len(x) for x in out_n))}, ch.S)
    for s in range(ch.S):
        T, mu = w.t[s // 2], w.mu[s % 2]
        zv = math.exp(mu / T) * T ** 1.5 * w.volume
        p = truncated_poisson(zv, w.n_max)
        mean_ref = float((np.arange(w.n_max + 1) * p).sum())
        m, se = batch_means(n_ser[:, s])
        assert abs(m - mean_ref) < 4 * se + 1e-9, (s, m, mean_ref, se)


def test_lj_mean_n_agrees_with_monte_carlo():
    w = W.small_lj(n_t=2, n_mu=2, n_max=14, mu=(-4.5, -3.0)).replace(sample_every=1)
    mc = oracle.Chain(w)
    mc.run(500)
    a = mc.run(8000)
    md = oracle.Chain(W.paper_schedule_md(w, x0=0.7, md_steps=5, md_dt=0.005, md_tau=0.05, sample_every=1))
    md.run(1000)
    b = md.run(12000)
    na, _ = per_state_series(a, mc.S)
    nb, _ = per_state_series(b, md.S)
    for s in range(mc.S):
        ma, sa = batch_means(na[:, s])
        mb, sb = batch_means(nb[:, s])
        assert abs(ma - mb) < 4 * math.hypot(sa, sb) + 1e-9, (s, ma, mb, sa, sb)
