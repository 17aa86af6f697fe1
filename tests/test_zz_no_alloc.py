"""regc_mbar_targets_static (the reweighted target averages with no allocation,
its intermediates in the library's fixed device array) against regc_mbar_targets on
the same solved handle: equal outputs on two calls in a row, the second with fewer
samples, states and targets (so the array still holds the first call's larger
contents), and a clear error beyond the stated limits."""
import sys

import numpy as np
import pytest

from paper_1908_11118_amd import regc
from paper_1908_11118_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def _samples(t, mu, n_max, per_state, seed):
    """Records of one sample per state: N Poisson around a state-dependent mean
    (clipped to 0..n_max), E = -2.5 N plus noise."""
    rng = np.random.default_rng(seed)
    S = len(t) * len(mu)
    lam = np.array([np.clip(np.exp(m / T + 6.0) * 0.02, 0.2, 0.8 * n_max) for T in t for m in mu])
    n = np.clip(rng.poisson(np.tile(lam, per_state)), 0, n_max).astype(np.int32)
    e = -2.5 * n + rng.normal(0.0, 1.0 + 0.1 * n)
    st = np.tile(np.arange(S, dtype=np.int32), per_state)
    return e, n, st


def _compare(mb, tt, tm):
    ref = mb.targets(tt, tm)
    got = mb.targets_static(tt, tm)
    for k in ("f", "mean_n", "mean_e", "mean_e2", "phase"):
        assert np.array_equal(got[k], ref[k]), (k, np.abs(got[k] - ref[k]).max())
    assert np.all(np.isfinite(got["mean_n"]))


def test_static_targets_match_on_two_calls_the_second_smaller():
    # first call: 8 x 8 states, 1.92e5 samples, 17 x 23 targets
    t1, mu1 = W.linear_grid(0.5, 2.0, 8), W.linear_grid(-8.0, -2.0, 8)
    e, n, st = _samples(t1, mu1, 40, 3000, seed=11)
    _say(f"[no-alloc] call 1: {len(e)} samples, 64 states, 17 x 23 targets")
    mb = regc.Mbar(t1, mu1, 40)
    mb.set_samples(e, n, st)
    _, conv, _, _ = mb.solve(tol=1e-10)
    assert conv
    _compare(mb, W.linear_grid(0.45, 2.1, 17), W.linear_grid(-8.5, -1.5, 23))
    # second call: 4 x 4 states, 1.6e4 samples, 5 x 7 targets
    t2, mu2 = W.linear_grid(0.7, 1.5, 4), W.linear_grid(-6.0, -3.0, 4)
    e2, n2, st2 = _samples(t2, mu2, 25, 1000, seed=12)
    _say(f"[no-alloc] call 2: {len(e2)} samples, 16 states, 5 x 7 targets")
    mb2 = regc.Mbar(t2, mu2, 25)
    mb2.set_samples(e2, n2, st2)
    _, conv, _, _ = mb2.solve(tol=1e-10)
    assert conv
    _compare(mb2, W.linear_grid(0.65, 1.6, 5), W.linear_grid(-6.5, -2.5, 7))
    # and the first handle again, after the smaller call
    _compare(mb, W.linear_grid(0.5, 2.0, 3), W.linear_grid(-7.0, -3.0, 2))
    # beyond the limits: 65 x 65 targets > 4096, rejected before any launch
    with pytest.raises(regc.RegcError) as ei:
        mb.targets_static(W.linear_grid(0.5, 2.0, 65), W.linear_grid(-8.0, -2.0, 65))
    assert ei.value.code == regc.EINVAL
    mb.close()
    mb2.close()


def test_static_targets_need_a_solution():
    t, mu = W.linear_grid(0.8, 1.2, 2), W.linear_grid(-5.0, -4.0, 2)
    e, n, st = _samples(t, mu, 10, 50, seed=3)
    mb = regc.Mbar(t, mu, 10)
    mb.set_samples(e, n, st)
    with pytest.raises(regc.RegcError) as ei:
        mb.targets_static(t, mu)
    assert ei.value.code == regc.ESTATE
    mb.close()
