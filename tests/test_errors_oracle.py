"""Pins of the oracle's error estimates of the reweighting (batch means at sampled
states, moving-block bootstrap at targets) and of the heat capacity and coverage.

The paper states no error estimator; these are the readings the project takes (batch
means of each state's series, a bootstrap over records with Philox-keyed block
starts, C = beta^2 var E at constant mu, theta = <N> / n_sites).  The pins fix them by
constructions whose answer is known exactly, by the single-state case (where the
reweighting is a plain weighted mean), by the analytic standard error of i.i.d.
samples, and by the ideal gas (E = 0, so C = 0)."""
import math

import numpy as np
import pytest

import oracle


def test_batch_means_of_a_constructed_series():
    # two states interleaved; state 0's series is 0,0,..,1,1,..,19,19 (batch b holds
    # value b), so the batch means are 0..19: mean 9.5, SE = sqrt(var(0..19)/20) with
    # var(0..19) = 35 (divisor 19)
    B, per = 20, 7
    s0 = np.repeat(np.arange(B), per)
    s1 = np.full(B * per, 4)
    state = np.empty(2 * B * per, dtype=np.int32)
    n = np.empty_like(state)
    state[0::2], n[0::2] = 0, s0
    state[1::2], n[1::2] = 1, s1
    mean, se = oracle.batch_means(3, state, n, B)
    assert mean[0] == 9.5 and abs(se[0] - math.sqrt(35.0 / 20.0)) < 1e-14
    assert mean[1] == 4.0 and se[1] == 0.0
    assert math.isnan(mean[2]) and math.isnan(se[2])          # no samples


def test_batch_means_uneven_batches_and_too_few_samples():
    # 41 samples in 4 batches: positions floor(b*41/4) .. -> batch sizes 10, 10, 10, 11
    # (a series whose batch means change when one sample moves between batches)
    x = np.arange(41) ** 2
    mean, se = oracle.batch_means(1, np.zeros(41, np.int32), x, 4)
    bm = [x[0:10].mean(), x[10:20].mean(), x[20:30].mean(), x[30:41].mean()]
    assert mean[0] == x.mean()
    assert abs(se[0] - np.std(bm, ddof=1) / 2.0) < 1e-12 * se[0]
    other = [x[0:11].mean(), x[11:21].mean(), x[21:31].mean(), x[31:41].mean()]
    assert abs(np.std(other, ddof=1) / 2.0 - se[0]) > 1e-3 * se[0]
    m2, s2 = oracle.batch_means(1, np.zeros(3, np.int32), np.arange(3), 4)
    assert math.isnan(m2[0]) and math.isnan(s2[0])


@pytest.mark.parametrize("R,block", [(50, 1), (50, 7), (37, 5), (64, 64)])
def test_bootstrap_multiplicities(R, block):
    for b in range(20):
        m = oracle.boot_multiplicity(R, block, b, 3)
        assert m.sum() == R and m.min() >= 0
        if block == R:
            assert np.all(m == 1)                  # one block holding every record
    # different replicates differ; the same replicate repeats
    assert not np.array_equal(oracle.boot_multiplicity(50, 1, 0, 3), oracle.boot_multiplicity(50, 1, 1, 3))
    assert np.array_equal(oracle.boot_multiplicity(50, 1, 4, 3), oracle.boot_multiplicity(50, 1, 4, 3))


def _one_state(R, rng):
    e = rng.normal(-30.0, 4.0, R)
    n = rng.poisson(12.0, R).astype(np.int32)
    return e, n


def test_single_state_bootstrap_is_the_resampled_mean():
    """With one state the reweighting weights are 1/n: each replicate's <N> is the
    multiplicity-weighted mean and C is beta^2 times the weighted variance; their
    spread over 400 replicates (blocks of one record) is the analytic standard error
    of the mean of i.i.d. samples within the bootstrap's own noise."""
    rng = np.random.default_rng(1)
    R = 400
    e, n = _one_state(R, rng)
    beta, lnz = np.array([1.0 / 1.3]), np.array([-2.0])
    nb = 400
    se_n, se_c, rn, rc, ok = oracle.mbar_bootstrap(beta, lnz, e, n, np.zeros(R, np.int32), 1, 1, nb, 9, [0.0],
                                                   beta, lnz, 60)
    assert ok
    for b in (0, 7, 399):
        m = oracle.boot_multiplicity(R, 1, b, 9).astype(float)
        wmean_n = (m * n).sum() / R
        wmean_e = (m * e).sum() / R
        wvar_e = (m * (e - wmean_e) ** 2).sum() / R
        assert abs(rn[b, 0] - wmean_n) < 1e-10 * abs(wmean_n)
        assert abs(rc[b, 0] - beta[0] ** 2 * wvar_e) < 1e-8 * beta[0] ** 2 * wvar_e
    analytic = n.std(ddof=1) / math.sqrt(R)
    assert abs(se_n[0] / analytic - 1.0) < 0.15        # relative noise of 400 replicates: ~3.5 %


def test_bootstrap_with_one_block_has_no_spread():
    rng = np.random.default_rng(2)
    R = 60
    e, n = _one_state(2 * R, rng)
    state = np.tile([0, 1], R).astype(np.int32)       # records of two samples, one per state
    beta = np.array([1.0, 0.8])
    lnz = np.array([-1.0, -1.5])
    f, logd, ok, _, _ = oracle.mbar_solve(beta, lnz, [R, R], e, n, tol=1e-12)
    assert ok
    se_n, se_c, rn, rc, ok = oracle.mbar_bootstrap(beta, lnz, e, n, state, 2, R, 5, 1, f, beta, lnz, 60, tol=1e-12)
    assert ok
    assert np.all(se_n < 1e-9) and np.all(se_c < 1e-9)


def test_longer_blocks_see_the_autocorrelation():
    """AR(1) series with phi = 0.9: the SE of the mean is about sqrt((1+phi)/(1-phi))
    = 4.4 times the i.i.d. value; blocks of one record miss it, blocks of 50 do not."""
    rng = np.random.default_rng(3)
    R, phi = 4000, 0.9
    x = np.zeros(R)
    for k in range(1, R):
        x[k] = phi * x[k - 1] + rng.normal()
    n = np.clip(np.rint(20 + 3 * x), 0, 60).astype(np.int32)
    e = -2.0 * n.astype(float)
    beta, lnz = np.array([1.0]), np.array([-1.0])
    args = (beta, lnz, e, n, np.zeros(R, np.int32), 1)
    s1 = oracle.mbar_bootstrap(*args, 1, 200, 5, [0.0], beta, lnz, 60)[0][0]
    s50 = oracle.mbar_bootstrap(*args, 50, 200, 5, [0.0], beta, lnz, 60)[0][0]
    assert s50 / s1 > 2.5


def test_heat_capacity_and_coverage():
    # single state: the reweighted <E^2> - <E>^2 is the population variance of E
    rng = np.random.default_rng(4)
    e, n = _one_state(500, rng)
    beta, lnz = np.array([1 / 0.7]), np.array([-3.0])
    f, logd, ok, _, _ = oracle.mbar_solve(beta, lnz, [500], e, n, tol=1e-12)
    t = oracle.mbar_targets(beta, lnz, e, n, logd, 60)
    hc, cov = oracle.heat_capacity_coverage(beta, t["mean_n"], t["mean_e"], t["mean_e2"], 64.0)
    assert abs(hc[0] - beta[0] ** 2 * np.var(e)) < 1e-8 * hc[0]
    assert abs(cov[0] - n.mean() / 64.0) < 1e-12
    # ideal gas: E = 0 in every sample, so C = 0 at every target
    nn = rng.poisson(5.0, 300).astype(np.int32)
    z = np.zeros(300)
    f, logd, ok, _, _ = oracle.mbar_solve([1.0, 0.5], [0.2, 0.1], [150, 150], z, nn, tol=1e-12)
    tt = oracle.mbar_targets([0.8, 1.7], [0.0, 0.3], z, nn, logd, 40)
    hc, _ = oracle.heat_capacity_coverage([0.8, 1.7], tt["mean_n"], tt["mean_e"], tt["mean_e2"], 1.0)
    assert np.all(hc == 0.0)
