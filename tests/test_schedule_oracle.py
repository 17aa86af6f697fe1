"""Pins of the oracle's paper schedule (the REGC step of Sec. II.A: a global coin
chooses a particle-exchange attempt per walker with probability x0, else a
replica-exchange step; then MC cycles of N displacements): the ideal-gas Poisson
law and the exact enumeration of an interacting lattice gas.  CPU only."""
import math

import numpy as np
import pytest

import oracle
from paper_1908_11118_amd import workloads as W
from tests.stats_util import batch_means, per_state_series, truncated_poisson
from tests.test_oracle_pins import _enumerate, _lattice_setup


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def test_step_structure():
    """One exchange attempt (trial 0) and mc_cycles * N displacements per walker and
    step; exchange steps at the coin's rate; samples every sample_every steps."""
    w = W.paper_schedule(W.small_lj(n_t=2, n_mu=2, n_max=12), x0=0.7, mc_cycles=3, sample_every=5)
    ch = oracle.Chain(w)
    out = ch.run(400, trace=True)
    st = ch.stats.sum(0)
    names = oracle.STAT_NAMES
    gc_att = st[names.index("ins_att")] + st[names.index("del_att")]
    steps_gc = gc_att // ch.S
    assert gc_att % ch.S == 0
    assert abs(steps_gc / 400 - 0.7) < 4 * math.sqrt(0.21 / 400)
    # exchange steps attempt every pair of their type: (1 - x0) * 400 steps happened
    assert ch.swap_att.sum() > 0
    assert st[names.index("ins_att")] > 0 and st[names.index("del_att")] > 0
    assert len(out["n"]) == (400 // 5) * ch.S
    assert out["bits"].shape == (400, ch.S, (1 + 3 * 12 + 31) // 32)
    # no trial index beyond 1 + mc_cycles * N was used
    for k in range(400):
        for wk in range(ch.S):
            bits = out["bits"][k, wk]
            top = max((32 * i + int(b).bit_length() - 1 for i, b in enumerate(bits) if b), default=0)
            assert top <= 3 * 12


def test_ideal_gas_poisson_paper_schedule():
    w = W.paper_schedule(W.ideal_gas(n_max=20), x0=0.8, mc_cycles=1, sample_every=1).replace(
        t=np.array([1.0, 1.5]), mu=np.array([-4.5, -3.5]))
    ch = oracle.Chain(w)
    ch.run(2000)
    out = ch.run(40000)
    n_ser, _ = per_state_series(out, ch.S)
    for s in range(ch.S):
        T, mu = w.t[s // 2], w.mu[s % 2]
        zv = math.exp(mu / T) * T ** 1.5 * w.volume
        p = truncated_poisson(zv, w.n_max)
        mean_ref = float((np.arange(w.n_max + 1) * p).sum())
        m, se = batch_means(n_ser[:, s])
        assert abs(m - mean_ref) < 4 * se + 1e-9, (s, m, mean_ref, se)


def test_lattice_gas_exact_enumeration_paper_schedule():
    box, slab, sites, eps_site, J = _lattice_setup()
    w = W.Workload(name="lattice", slab=slab, lx=box, ly=box, zlo=0.0, zhi=4.0,
                   t=np.array([0.8, 1.2]), mu=np.array([-4.2, -3.4]), n_max=len(sites), mode=2,
                   sites=sites, schedule=1, x0=0.9, mc_cycles=2, sample_every=1)
    ch = oracle.Chain(w)
    ch.run(3000)
    out = ch.run(60000)
    n_ser, _ = per_state_series(out, ch.S)
    for s in range(ch.S):
        T, mu = w.t[s // 2], w.mu[s % 2]
        ref, _ = _enumerate(eps_site, J, T, mu)
        m, se = batch_means(n_ser[:, s])
        assert abs(m - ref) < 4 * se + 1e-9, (s, m, ref, se)
