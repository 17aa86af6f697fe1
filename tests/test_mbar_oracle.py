"""Pins of the oracle's multistate reweighting: the single-state limit, the
fixed-point identities, the ideal-gas closed form, invariances and exact
lattice-gas enumeration at an unsampled state.  CPU only."""
import math

import numpy as np
import pytest

import oracle
from paper_1908_11118_amd import workloads as W
from tests.stats_util import per_state_series, truncated_poisson
from tests.test_oracle_pins import _enumerate, _lattice_setup


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def test_single_state_is_plain_average():
    rng = np.random.default_rng(1)
    e = rng.normal(-20, 5, 5000)
    n = rng.integers(0, 30, 5000).astype(np.int32)
    f, logd, ok, it, _ = oracle.mbar_solve([1.3], [0.2], [5000], e, n)
    assert ok and f[0] == 0.0
    r = oracle.mbar_targets([1.3], [0.2], e, n, logd, 40)
    assert abs(r["mean_n"][0] - n.mean()) < 1e-10
    assert abs(r["mean_e"][0] - e.mean()) < 1e-9
    assert abs(r["p_n"][0].sum() - 1) < 1e-12
    assert abs(r["f"][0]) < 1e-10


def _ideal_samples(rng, Ts, mus, V, n_max, per_state):
    beta, lnz, omega, ns = [], [], [], []
    for T in Ts:
        for mu in mus:
            zv = math.exp(mu / T) * T ** 1.5 * V
            p = truncated_poisson(zv, n_max)
            ns.append(rng.choice(n_max + 1, size=per_state, p=p))
            beta.append(1 / T)
            lnz.append(oracle.state_lnz(T, mu))
            omega.append(per_state)
    n = np.concatenate(ns).astype(np.int32)
    return np.array(beta), np.array(lnz), np.array(omega), np.zeros(len(n)), n


def _xi(T, mu, V, n_max):
    zv = math.exp(mu / T) * T ** 1.5 * V
    k = np.arange(n_max + 1)
    logt = k * math.log(zv) - np.array([math.lgamma(i + 1) for i in k])
    m = logt.max()
    return m + math.log(np.exp(logt - m).sum())


def test_ideal_gas_free_energies_and_unsampled_mean():
    rng = np.random.default_rng(2)
    Ts, mus, V, n_max = [1.0, 1.3], [-4.6, -4.0, -3.4], 288.0, 40
    beta, lnz, omega, e, n = _ideal_samples(rng, Ts, mus, V, n_max, 20000)
    f, logd, ok, it, _ = oracle.mbar_solve(beta, lnz, omega, e, n, tol=1e-11)
    assert ok
    k = 0
    for T in Ts:
        for mu in mus:
            ref = -(_xi(T, mu, V, n_max) - _xi(Ts[0], mus[0], V, n_max))
            assert abs(f[k] - ref) < 0.02, (k, f[k], ref)
            k += 1
    # unsampled state inside the grid: truncated-Poisson mean
    T, mu = 1.15, -3.7
    r = oracle.mbar_targets([1 / T], [oracle.state_lnz(T, mu)], e, n, logd, n_max)
    zv = math.exp(mu / T) * T ** 1.5 * V
    p = truncated_poisson(zv, n_max)
    mean_ref = float((np.arange(n_max + 1) * p).sum())
    assert abs(r["mean_n"][0] - mean_ref) < 0.02 * mean_ref
    assert np.abs(r["p_n"][0] - p).sum() < 0.02
    assert r["phase"][0] == int(np.argmax(p))


def test_fixed_point_identities_and_invariances():
    rng = np.random.default_rng(3)
    S = 6
    beta = 1 / np.array([0.8, 0.8, 0.8, 1.4, 1.4, 1.4])
    lnz = np.array([-3.0, -2.5, -2.0, -2.8, -2.3, -1.9])
    omega = np.array([700, 800, 900, 600, 750, 650])
    ns = omega.sum()
    n = rng.integers(0, 12, ns).astype(np.int32)
    e = -1.5 * n + rng.normal(0, 2.0, ns)
    f, logd, ok, it, _ = oracle.mbar_solve(beta, lnz, omega, e, n, tol=1e-12)
    assert ok
    u = beta[:, None] * e[None, :] - n[None, :] * lnz[:, None]
    w = np.exp(f[:, None] - u - logd[None, :])
    assert np.allclose(w.sum(1), 1.0, atol=1e-9)              # each state's weights normalise
    assert np.allclose((omega[:, None] * w).sum(0), 1.0, atol=1e-9)  # sum_k Omega_k w_n(k) = 1
    # permutation of the samples
    perm = rng.permutation(ns)
    f2, _, ok2, _, _ = oracle.mbar_solve(beta, lnz, omega, e[perm], n[perm], tol=1e-12)
    assert ok2 and np.allclose(f2, f, atol=1e-9)
    # constant added to every energy: f_s shifts by beta_s c (gauge-fixed at state 0)
    c = 7.5
    f3, logd3, ok3, _, _ = oracle.mbar_solve(beta, lnz, omega, e + c, n, tol=1e-12)
    assert ok3 and np.allclose(f3, f + (beta - beta[0]) * c, atol=1e-8)
    r1 = oracle.mbar_targets([1 / 1.1], [-2.4], e, n, logd, 20)
    r3 = oracle.mbar_targets([1 / 1.1], [-2.4], e + c, n, logd3, 20)
    assert abs(r1["mean_n"][0] - r3["mean_n"][0]) < 1e-9
    assert abs(r1["mean_e"][0] + c - r3["mean_e"][0]) < 1e-8
    # one application of the map at the solution returns the solution
    fo, _ = oracle.mbar_iterate(beta, lnz, omega, e, n, f)
    assert np.allclose(fo - fo[0], f, atol=1e-10)


def test_lattice_gas_reweighting_to_unsampled_state():
    box, slab, sites, eps_site, J = _lattice_setup()
    t = np.array([0.8, 1.0, 1.2])
    mu = np.array([-4.4, -3.9, -3.4])
    w = W.Workload(name="lattice", slab=slab, lx=box, ly=box, zlo=0.0, zhi=4.0, t=t, mu=mu,
                   n_max=len(sites), mode=2, sites=sites, swap_every=10, sample_every=5, n_sweeps=40000)
    ch = oracle.Chain(w)
    ch.run(2000)
    out = ch.run(w.n_sweeps)
    beta, lnz = oracle.state_arrays(w)
    omega = np.bincount(out["state"], minlength=ch.S)
    targets = [(0.9, -3.65), (1.1, -4.15), (1.2, -3.0)]
    tb = [1 / T for T, _ in targets]
    tz = [oracle.state_lnz(T, m, mode=2) for T, m in targets]
    f, logd, ok, _, _ = oracle.mbar_solve(beta, lnz, omega, out["e"], out["n"], tol=1e-10)
    assert ok
    full = oracle.mbar_targets(tb, tz, out["e"], out["n"], logd, len(sites))
    # block estimates for the standard error
    n_ser, e_ser = per_state_series(out, ch.S)
    B = 10
    m = len(n_ser) // B
    blocks = []
    for b in range(B):
        nb = n_ser[b * m:(b + 1) * m].ravel()
        eb = e_ser[b * m:(b + 1) * m].ravel()
        om = np.full(ch.S, m)
        st = np.tile(np.arange(ch.S), m)
        order = np.argsort(st, kind="stable")
        fb, ldb, okb, _, _ = oracle.mbar_solve(beta, lnz, om, eb[order], nb[order], tol=1e-9)
        blocks.append(oracle.mbar_targets(tb, tz, eb[order], nb[order], ldb, len(sites))["mean_n"])
    se = np.array(blocks).std(0, ddof=1) / math.sqrt(B)
    for k, (T, muv) in enumerate(targets):
        ref, _ = _enumerate(eps_site, J, T, muv)
        assert abs(full["mean_n"][k] - ref) < 4 * se[k] + 1e-3, (k, full["mean_n"][k], ref, se[k])
