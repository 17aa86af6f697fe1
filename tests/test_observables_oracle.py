"""Pins of the oracle's reweighted structural observables (Sec. III.A: axial density
in z bins and the lateral pair distribution of a layer; Sec. II.B, Eq. (11) for
their reweighted averages): brute-force counts with explicit periodic images,
single-state reweighting identities, and ideal-gas closed forms (flat density,
annulus areas) at an unsampled state.  CPU only."""
import math

import numpy as np
import pytest

import oracle
from paper_1908_11118_amd import workloads as W
from tests.stats_util import truncated_poisson

SPEC = dict(dz=0.12, layer=(0.6, 1.6), dr=0.1, nr=28)


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def _brute(xyz, w, spec):
    nz = int(math.ceil((w.zhi - w.zlo) / spec["dz"]))
    edges = w.zlo + spec["dz"] * np.arange(nz + 1)
    zc, _ = np.histogram(xyz[:, 2], bins=edges)
    lo, hi = spec["layer"]
    lay = xyz[(xyz[:, 2] >= lo) & (xyz[:, 2] < hi)]
    d = []
    for i in range(len(lay)):
        for j in range(i + 1, len(lay)):
            best = min(math.hypot(lay[i, 0] - lay[j, 0] + a * w.lx, lay[i, 1] - lay[j, 1] + b * w.ly)
                       for a in (-1, 0, 1) for b in (-1, 0, 1))
            d.append(best)
    rc, _ = np.histogram(d, bins=spec["dr"] * np.arange(spec["nr"] + 1))
    return np.concatenate([zc, rc, [len(lay)]]).astype(float)


def test_observables_of_a_configuration_match_brute_force():
    w = W.config1()
    ch = oracle.Chain(w, observables=SPEC)
    rng = np.random.default_rng(1)
    for n in (0, 1, 2, 25, 40):
        xyz = np.column_stack([rng.uniform(0, w.lx, n), rng.uniform(0, w.ly, n), rng.uniform(w.zlo, w.zhi, n)])
        if n >= 2:
            xyz[1] = [xyz[0, 0] + 2.9, xyz[0, 1] - 0.4, 1.0]     # a pair across the periodic boundary
            xyz[0, 2] = 1.1
        got = ch.observables(xyz)
        assert np.array_equal(got, _brute(xyz, w, SPEC)), n
    # a particle exactly at z_hi falls in the last bin
    got = ch.observables(np.array([[1.0, 1.0, w.zhi]]))
    nz = int(math.ceil((w.zhi - w.zlo) / SPEC["dz"]))
    assert got[nz - 1] == 1.0


def test_single_state_reweighting_gives_sample_means():
    w = W.small_lj(n_t=1, n_mu=1, n_max=12).replace(swap_every=0)
    ch = oracle.Chain(w, observables=SPEC)
    ch.run(200)
    out = ch.run(2000)
    beta, lnz = oracle.state_arrays(w)
    f, logd, ok, _, _ = oracle.mbar_solve(beta, lnz, [len(out["e"])], out["e"], out["n"])
    assert ok
    mean, cond = oracle.mbar_observables(beta, lnz, out["e"], out["n"], logd, w.n_max, out["obs"])
    assert np.allclose(mean[0], out["obs"].mean(0), rtol=1e-10, atol=1e-12)
    for N in np.unique(out["n"]):
        sel = out["n"] == N
        assert np.allclose(cond[0, N], out["obs"][sel].mean(0), rtol=1e-10, atol=1e-12)
    # mean = sum over phases of p(N) times the conditional average
    pn = oracle.mbar_targets(beta, lnz, out["e"], out["n"], logd, w.n_max)["p_n"][0]
    assert np.allclose((pn[:, None] * cond[0]).sum(0), mean[0], rtol=1e-10, atol=1e-12)


def test_ideal_gas_profiles_at_an_unsampled_state():
    w = W.ideal_gas(n_max=30).replace(t=np.array([1.0, 1.4]), mu=np.array([-4.6, -4.0]), n_sweeps=6000)
    spec = dict(dz=1.0, layer=(2.0, 6.0), dr=0.25, nr=10)
    ch = oracle.Chain(w, observables=spec)
    ch.run(300)
    out = ch.run(w.n_sweeps)
    beta, lnz = oracle.state_arrays(w)
    omega = np.bincount(out["state"], minlength=ch.S)
    f, logd, ok, _, _ = oracle.mbar_solve(beta, lnz, omega, out["e"], out["n"])
    assert ok
    T, mu = 1.2, -4.3
    tb, tz = np.array([1.0 / T]), np.array([oracle.state_lnz(T, mu)])
    mean, _ = oracle.mbar_observables(tb, tz, out["e"], out["n"], logd, w.n_max, out["obs"])
    zv = math.exp(mu / T) * T ** 1.5 * w.volume
    p = truncated_poisson(zv, w.n_max)
    k = np.arange(w.n_max + 1)
    mean_n = float((k * p).sum())
    nz = 8
    # flat axial density: each unit-height bin holds <N> / 8 on average
    assert np.allclose(mean[0, :nz], mean_n / nz, rtol=0.05)
    # layer pairs by lateral distance: proportional to annulus areas (r < L/2)
    pairs = mean[0, nz:nz + 10]
    r = spec["dr"] * np.arange(11)
    area = math.pi * (r[1:] ** 2 - r[:-1] ** 2)
    # E[pairs in bin] = E[N_l (N_l - 1)] / 2 * area / A, N_l ~ Binomial(N, 4/8)
    en2 = float((k * (k - 1) * p).sum()) * 0.25
    ref = 0.5 * en2 * area / (w.lx * w.ly)
    assert np.allclose(pairs[3:].sum(), ref[3:].sum(), rtol=0.08)
    assert abs(mean[0, -1] - mean_n * 0.5) < 0.05 * mean_n
