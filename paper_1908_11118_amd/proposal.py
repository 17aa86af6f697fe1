"""The learned insertion proposal end to end: training data captured from plain
REGC runs on the GPU, training of the proposal network on the GPU, and the
comparison of wall time to a target accuracy of <N>(T, mu) with and without it.

Training data (a reading: the network's inputs are the occupancy only): the
sweep-end configurations of every walker of plain runs, as voxel lists on the
device.  Training example: one configuration, one of its particles left out;
input the occupancy of the others, target the left-out particle's voxel;
cross-entropy loss, Adam.

Time to accuracy (a reading of "wall-s to <N>(T, mu) at 3 SE"): both forms start
from the same equilibrated state; after every chunk of sweeps the per-state mean
N and its batch-means standard error are computed from all samples so far; the
form has reached the target at the first chunk where (a) every state's standard
error is at most tau particles, (b) at least `frac` of the states lie within
3 sqrt(SE^2 + SE_ref^2) of the long reference run and (c) the mean squared
z-score is at most 1.3.  Only the GPU sampling time (launches to synchronisation)
is counted.
"""
from __future__ import annotations

import time
from typing import Dict, Optional

import numpy as np

from . import regc
from . import workloads as W


def capture_dataset(workload, seeds=(1, 2), burnin: int = 2000, sweeps: int = 10000, every: int = 1,
                    precision: int = regc.FP32PAIR):
    """Device data set of sweep-end configurations of plain runs: returns torch
    tensors vox [n_examples][n_max] (int16 storage of uint16 voxel indices) and
    n [n_examples] (int32), n_examples = len(seeds) * (sweeps // every) * S."""
    import torch
    w0 = workload.replace(sample_every=0)
    S, nmax = w0.n_states, w0.n_max
    per = sweeps // every
    vox = torch.zeros((len(seeds) * per * S, nmax), dtype=torch.int16, device="cuda")
    n = torch.zeros((len(seeds) * per * S,), dtype=torch.int32, device="cuda")
    off = 0
    for seed in seeds:
        with regc.Regc(w0.replace(seed=seed), precision=precision, sample_capacity=0) as g:
            g.run(burnin)
            for _ in range(per):
                g.run(every)
                g.capture_voxels(vox[off].data_ptr(), n[off].data_ptr())
                off += S
            g.sync()
    return vox, n


def capture_batch(classes, burnin: int = 2000, sweeps: int = 500, seed: int = 1, precision: int = regc.FP32PAIR,
                  **opts):
    """Per-class device data sets of sweep-end configurations of a plain uneven
    batch: returns [(vox, n)] per class (torch tensors as in capture_dataset, rows of
    the class's walkers only, n_max the largest over the batch) and the checkpoint
    of the batch after burn-in."""
    import torch
    wl = [w.replace(sample_every=0, seed=seed) for w in classes]
    with regc.Regc(wl, precision=precision, sample_capacity=0, **opts) as g:
        g.run(burnin)
        blob = g.checkpoint()
        Wa, nmax = g.W, max(w.n_max for w in wl)
        vox = torch.zeros((sweeps * Wa, nmax), dtype=torch.int16, device="cuda")
        n = torch.zeros((sweeps * Wa,), dtype=torch.int32, device="cuda")
        for s in range(sweeps):
            g.run(1)
            g.capture_voxels(vox[s * Wa].data_ptr(), n[s * Wa].data_ptr())
        g.sync()
        offs, cnts = g.offsets, g.counts
    out = []
    for o, c in zip(offs, cnts):
        rows = (torch.arange(sweeps, device="cuda")[:, None] * Wa + o + torch.arange(c, device="cuda")[None, :])
        rows = rows.reshape(-1)
        out.append((vox[rows].contiguous(), n[rows].contiguous()))
    del vox, n
    return out, blob


def train(vox, n, steps: int = 10000, batch: int = 256, lr: float = 1e-3, seed: int = 100, init_seed: int = 0,
          report_every: int = 500, log=None) -> "regc.Mlp":
    """Trains a fresh network on the device data set; returns it (regc.Mlp)."""
    net = regc.Mlp(W.mlp_pack(W.mlp_init(init_seed)))
    nmax = int(vox.shape[1])
    done = 0
    while done < steps:
        k = min(report_every, steps - done)
        loss = net.train(int(vox.shape[0]), nmax, vox.data_ptr(), n.data_ptr(), steps=k, batch=batch, lr=lr,
                         seed=seed + done)
        done += k
        if log:
            log(f"[train] step {done} loss {loss:.4f}")
    return net


def reference(workload, sweeps: int = 100000, burnin: int = 2000, seed: int = 4, precision: int = regc.FP64,
              chunk: int = 5000):
    """Long plain run: per-state mean N and its standard error (records every sweep)."""
    w = workload.replace(seed=seed, sample_every=1)
    S = w.n_states
    series = _Series(S)
    with regc.Regc(w, precision=precision, sample_capacity=chunk * S) as g:
        g.run(burnin)
        g.clear_samples()
        done = 0
        while done < sweeps:
            k = min(chunk, sweeps - done)
            g.run(k)
            smp = g.samples()
            series.add(smp["state"], smp["n"])
            g.clear_samples()
            done += k
    return series.mean_se()


class _Series:
    """All (state, N) samples of a run so far, in sample order; their per-state mean
    and batch-means standard error come from the library (regc_batch_means)."""

    def __init__(self, S: int, n_batches: int = 20):
        self.S, self.nb = S, n_batches
        self.state = np.zeros(1 << 16, np.int32)
        self.n = np.zeros(1 << 16, np.int32)
        self.L = 0

    def add(self, state, n):
        k = len(n)
        while self.L + k > len(self.n):
            self.state = np.concatenate([self.state, np.zeros_like(self.state)])
            self.n = np.concatenate([self.n, np.zeros_like(self.n)])
        self.state[self.L:self.L + k] = state
        self.n[self.L:self.L + k] = n
        self.L += k

    def mean_se(self):
        """Mean and SE per state (SE infinite below n_batches samples)."""
        if self.L == 0:
            return np.full(self.S, np.nan), np.full(self.S, np.inf)
        m, se = regc.batch_means(self.state[:self.L], self.n[:self.L], self.S, self.nb)
        return m, np.where(np.isnan(se), np.inf, se)


def time_to_accuracy(workload, blob: bytes, ref_mean, ref_se, net: Optional["regc.Mlp"] = None,
                     alpha: float = 0.0, precision: int = regc.FP32PAIR, chunk: int = 250,
                     max_sweeps: int = 200000, max_seconds: float = 1e9, tau: float = 0.1, frac: float = 0.98,
                     max_chi2: float = 1.3, seed: int = 3, hold: int = 3, log=None) -> Dict:
    """Runs from the checkpoint `blob` (written by equilibrated_state with the same
    seed) until the accuracy target is met or max_sweeps / max_seconds of GPU time
    are spent; returns {"t_acc_s", "sweeps", "reached", "max_se", "frac_within",
    "chi2", "ins_acc", ...}.  (Sweeps are REGC steps for the paper's schedule.)  The
    target is checked after every `chunk` sweeps up to 16 chunks, then every
    sixteenth of the sweeps so far (rounded to chunks), so that long runs check it
    about a hundred times.  It counts as met when it holds at `hold` consecutive
    checks (the time is that of the last of them): the batch-means errors of a short
    run are noisy, and the first check that happens to pass would make the time
    depend on that noise more than on the sampler."""
    w = workload.replace(seed=seed, sample_every=1)
    S = w.n_states
    series = _Series(S)
    t_gpu = 0.0
    res = {"reached": False}
    with regc.Regc(w, precision=precision, sample_capacity=chunk * S) as g:
        g.restore(blob)
        g.clear_samples()
        if net is not None and alpha > 0:
            g.set_proposal(net, alpha)
        st0 = g.stats()["stats"].copy()
        done, next_check, checks, streak = 0, chunk, 0, 0
        while done < max_sweeps:
            g.sync()
            t0 = time.perf_counter()
            g.run(chunk)
            g.sync()
            t_gpu += time.perf_counter() - t0
            done += chunk
            smp = g.samples()
            g.clear_samples()
            series.add(smp["state"], smp["n"])
            if done < next_check and done < max_sweeps and t_gpu < max_seconds:
                continue
            next_check = done + max(chunk, (done // 16) // chunk * chunk)
            checks += 1
            m, se = series.mean_se()
            z = (m - ref_mean) / np.sqrt(se ** 2 + ref_se ** 2)
            within = float(np.mean(np.abs(z) <= 3.0))
            chi2 = float(np.mean(z ** 2))
            ok = bool(np.all(se <= tau) and within >= frac and chi2 <= max_chi2)
            streak = streak + 1 if ok else 0
            res = {"reached": streak >= hold, "t_acc_s": t_gpu, "sweeps": done, "max_se": float(np.max(se)),
                   "frac_within": within, "chi2": chi2}
            if log and checks % 10 == 0:
                log(f"[t_acc] alpha={alpha} sweeps={done} t={t_gpu:.2f}s max_se={res['max_se']:.3f} "
                    f"within={within:.3f} chi2={chi2:.2f}")
            if res["reached"] or t_gpu >= max_seconds:
                break
        res["se_by_state"] = se.tolist()
        res["mean_by_state"] = m.tolist()
        st = g.stats()["stats"] - st0
        res["ins_acc"] = float(st[:, 3].sum() / max(1, st[:, 2].sum()))
        res["ins_acc_by_state"] = (st[:, 3] / np.maximum(st[:, 2], 1)).tolist()
        res["ms_per_sweep"] = 1e3 * t_gpu / max(done, 1)
        if net is not None and alpha > 0:
            res["proposal"] = g.proposal_stats()
    res["alpha"] = alpha
    return res


def equilibrated_state(workload, seed: int = 3, burnin: int = 2000, precision: int = regc.FP32PAIR) -> bytes:
    """Checkpoint of a plain run after burn-in: the common starting point."""
    with regc.Regc(workload.replace(seed=seed, sample_every=0), precision=precision, sample_capacity=0) as g:
        g.run(burnin)
        return g.checkpoint()


def efficiency_ratio(plain: Dict, learned: Dict, min_se: float = 1e-3) -> Dict:
    """Per-state statistical efficiency 1 / (SE^2 t) of the learned form over the
    plain form, from the end of two time_to_accuracy runs (states whose standard
    error is below min_se in either run -- frozen at 0 or at the cap -- are left
    out).  Returns the median, minimum and maximum ratio and the state count."""
    sp = np.asarray(plain["se_by_state"])
    sl = np.asarray(learned["se_by_state"])
    ok = (sp > min_se) & (sl > min_se) & np.isfinite(sp) & np.isfinite(sl)
    if not ok.any():
        return {"states": 0}
    r = (sp[ok] ** 2 * plain["t_acc_s"]) / (sl[ok] ** 2 * learned["t_acc_s"])
    return {"states": int(ok.sum()), "median": float(np.median(r)), "min": float(r.min()), "max": float(r.max()),
            "geomean": float(np.exp(np.mean(np.log(r))))}
