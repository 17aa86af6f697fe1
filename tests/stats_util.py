"""Statistics helpers and independent reference formulas used by the pins."""
import math

import numpy as np


def batch_means(x, n_batches=20):
    """Mean and its standard error from n_batches contiguous batch means."""
    x = np.asarray(x, dtype=np.float64)
    m = len(x) // n_batches
    b = x[: m * n_batches].reshape(n_batches, m).mean(axis=1)
    return float(x.mean()), float(b.std(ddof=1) / math.sqrt(n_batches))


def truncated_poisson(lam, n_max):
    """pmf of a Poisson(lam) restricted to 0..n_max (log-space)."""
    k = np.arange(n_max + 1)
    logp = k * math.log(lam) - np.array([math.lgamma(i + 1) for i in k])
    logp -= logp.max()
    p = np.exp(logp)
    return p / p.sum()


def per_state_series(samples, S):
    """Rearrange flat samples (recorded S at a time, walker order) into per-state
    time series [n_records, S] of N and E."""
    st = samples["state"].reshape(-1, S)
    n = samples["n"].reshape(-1, S)
    e = samples["e"].reshape(-1, S)
    order = np.argsort(st, axis=1)
    return (np.take_along_axis(n, order, axis=1), np.take_along_axis(e, order, axis=1))


def lj_ts(r2, eps, sig, rc):
    """Truncated-shifted LJ 12-6 written with powers of r (numpy, vectorised)."""
    r = np.sqrt(r2)
    v = 4 * eps * ((sig / r) ** 12 - (sig / r) ** 6) - 4 * eps * ((sig / rc) ** 12 - (sig / rc) ** 6)
    return np.where(r < rc, v, 0.0)


def energy_image_sum(xyz, slab, lx, ly, eps_gg=1.0, sig_gg=1.0, eps_gs=1.0, sig_gs=1.0, rc=2.5):
    """Brute-force total energy: explicit sum over periodic images -1..1 in x and y
    (no minimum-image convention), gas-gas once per pair, gas-slab for every atom."""
    xyz = np.asarray(xyz).reshape(-1, 3)
    slab = np.asarray(slab).reshape(-1, 3)
    shifts = np.array([[a * lx, b * ly, 0.0] for a in (-1, 0, 1) for b in (-1, 0, 1)])
    e = 0.0
    n = len(xyz)
    for i in range(n):
        for j in range(i + 1, n):
            d = xyz[i] - (xyz[j] + shifts)
            e += lj_ts((d * d).sum(1), eps_gg, sig_gg, rc).sum()
        if len(slab):
            d = xyz[i][None, None, :] - (slab[:, None, :] + shifts[None, :, :])
            e += lj_ts((d * d).sum(2), eps_gs, sig_gs, rc).sum()
    return float(e)


def assert_within_3se(z, label=""):
    """The 3-standard-error bar over several states: every |z| <= 4, at most
    max(1, 5 %) of the states beyond 3 (under the null each exceeds 3 with about
    0.3-0.5 % probability with 20-batch errors), and a mean z^2 no larger than the
    99.99 % point of chi^2 with as many degrees of freedom as states, per state."""
    from scipy.stats import chi2
    z = np.asarray(z, dtype=np.float64)
    k = len(z)
    beyond = int(np.sum(np.abs(z) > 3.0))
    msg = f"{label}: z = {np.round(z, 2).tolist()}"
    assert np.all(np.abs(z) <= 4.0), msg
    assert beyond <= max(1, int(round(0.05 * k))), msg
    assert float(np.mean(z * z)) <= chi2.ppf(0.9999, k) / k, msg
