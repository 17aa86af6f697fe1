"""Pins of the oracle's aiAT@REGC ingredients (Sec. III.A, Eq. (12)): the lowest
recorded energy per N against the samples themselves, the stored configuration's
recomputed energy, and the phase map's switching points for a convex E_min(N)
(phase N -> N+1 exactly at mu = E_min(N+1) - E_min(N)).  CPU only."""
import numpy as np
import pytest

import oracle
from paper_1908_11118_amd import workloads as W


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def test_minima_are_the_lowest_recorded_samples():
    w = W.config1()
    ch = oracle.Chain(w)
    out = ch.run(400)
    for N in range(w.n_max + 1):
        sel = out["n"] == N
        if sel.any():
            assert ch.min_e[N] == out["e"][sel].min()
            e_rec = ch.energy(ch.min_xyz[N, :N])
            assert abs(e_rec - ch.min_e[N]) <= 1e-9 * max(1.0, abs(e_rec))
            x = ch.min_xyz[N, :N]
            assert np.all((x[:, 0] >= 0) & (x[:, 0] < w.lx) & (x[:, 2] >= w.zlo) & (x[:, 2] <= w.zhi))
        else:
            assert ch.min_e[N] == np.inf
    # more sampling never raises a minimum
    before = ch.min_e.copy()
    ch.run(100)
    assert np.all(ch.min_e <= before)


def test_aiat_phase_switches_at_the_energy_slopes():
    N = np.arange(9)
    e = -3.0 * N + 0.25 * N * N          # convex: slopes -2.75, -2.25, ...
    e[5] = np.inf                        # a never-recorded N is skipped
    mu_switch = [e[k + 1] - e[k] for k in range(4)]
    eps = 1e-9
    for k, m in enumerate(mu_switch):
        below, above = oracle.aiat_phase(e, [m - eps, m + eps])
        assert below == k and above == k + 1
    # past N = 4 the next recorded phase is 6: switch at (e[6] - e[4]) / 2
    m = 0.5 * (e[6] - e[4])
    assert list(oracle.aiat_phase(e, [m - eps, m + eps])) == [4, 6]
    assert oracle.aiat_phase(e, [-100.0])[0] == 0 and oracle.aiat_phase(e, [100.0])[0] == 8
