"""Launch-shape autotuner for REGC sampling contexts.

The choices it makes -- walkers per workgroup, wavefronts per walker, batched
trials, the cull pass, slab column binning and its column width (the slab's cell
size), sweeps per launch, graph replay of several exchange intervals per submission
persistent launches of several intervals, and the walker order dealt by particle count
(which wave runs which walker) -- change only the order of floating-point sums, never
the chain (FP64 trajectories are identical for every choice), so the tuned run
samples the same distribution.

Procedure: equilibrate one context with default options, checkpoint it, then for
each candidate build a context, restore the checkpoint, run a short timed window
and keep the fastest.  The search starts from the library's own choices and is
greedy over one option at a time.  Results are cached in a JSON file keyed by the
workload signature and the device name.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time
from typing import Dict, List, Optional

from . import regc

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "regc_autotune.json")


def _signature(workloads, precision: int) -> str:
    parts = []
    for w in workloads:
        parts.append(f"{len(w.slab)}:{w.lx}:{w.ly}:{w.zhi - w.zlo}:{w.n_max}:{len(w.t)}x{len(w.mu)}:"
                     f"{w.trials}:{w.swap_every}:{w.mode}")
    dev = "unknown"
    try:
        import torch
        if torch.cuda.is_available():
            dev = torch.cuda.get_device_name(0)
    except Exception:
        pass
    key = f"{precision}|{dev}|" + "|".join(parts)
    return hashlib.sha1(key.encode()).hexdigest()[:16]


def _measure(workloads, precision: int, blob: bytes, opts: Dict, sweeps: int) -> float:
    # with graph replay, one whole replay period (graph_intervals exchange intervals)
    # is run before timing, so that the capture happens outside the timed region,
    # and at least two periods are timed
    period = workloads[0].swap_every * max(1, opts.get("graph_intervals", 0))
    sweeps = max(sweeps, 2 * period)
    with regc.Regc(workloads, precision=precision, sample_capacity=0, **opts) as g:
        g.restore(blob)
        g.run(period)                           # first launches: graph capture, caches
        g.sync()
        t0 = time.perf_counter()
        g.run(sweeps)
        g.sync()
        dt = time.perf_counter() - t0
    trials = sweeps * sum(w.n_states * w.trials for w in workloads)
    return trials / dt


def autotune(workloads, precision: int = regc.FP32PAIR, warm_sweeps: int = 500, measure_sweeps: int = 40,
             cache_path: Optional[str] = DEFAULT_CACHE, verbose: bool = False) -> Dict:
    """Returns {"options": best option dict, "trials_per_s": rate, "table": [...]}."""
    wl = list(workloads) if isinstance(workloads, (list, tuple)) else [workloads]
    sig = _signature(wl, precision)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            cache = json.load(open(cache_path))
        except (OSError, ValueError):
            cache = {}
        if sig in cache:
            return cache[sig]
    interval = wl[0].swap_every
    measure_sweeps = max(interval, (measure_sweeps // max(interval, 1)) * max(interval, 1))
    with regc.Regc(wl, precision=precision, sample_capacity=0) as g:
        g.run(warm_sweeps)
        blob = g.checkpoint()
    table: List[Dict] = []

    def trial(opts):
        try:
            rate = _measure(wl, precision, blob, opts, measure_sweeps)
        except regc.RegcError as err:        # a shape this device or workload cannot run
            if err.code not in (regc.EUNSUPPORTED, regc.EINVAL):
                raise
            rate = 0.0
        table.append({"options": dict(opts), "trials_per_s": rate})
        if verbose:
            print(f"[autotune] {opts} -> {rate:.4g} trials/s", file=sys.stderr, flush=True)
        return rate

    # 0 everywhere: the library's own choices
    best = {"walkers_per_block": 0, "split": 0, "batch_trials": 0, "cull": 0, "slab_bins": 0, "slab_cell": 0.0,
            "sweeps_per_launch": 0, "graph_intervals": 0, "persistent": 0, "balance": 0}
    best_rate = trial(best)
    spl = sorted({s for s in (interval // 2, max(1, interval // 5)) if 0 < s < interval})
    # batched trials: (trials per batch, waves per walker) -- one wave per walker, or one
    # wave per trial
    space = [("walkers_per_block", [1, 2, 4, 8]), ("split", [1, 2, 4]), ("batch", [(2, 1), (4, 1), (2, 2), (4, 4)]),
             ("cull", [1]), ("slab_bins", [-1]), ("slab_cell", [1.25, 1.5]), ("sweeps_per_launch", spl),
             ("graph_intervals", [4, 10]), ("persistent", [10]), ("balance", [1, -1])]
    for name, values in space:
        for v in values:
            cand = dict(best)
            if name == "batch":
                cand["batch_trials"], cand["split"], cand["cull"] = v[0], v[1], 0
                if v[1] > 1:
                    cand["walkers_per_block"] = 1
            else:
                cand[name] = v
            if name == "split" and v > 1:
                cand["batch_trials"], cand["walkers_per_block"] = 1, 1
            if name == "persistent":
                # whole exchange intervals in one cooperative launch: no graph, cull or batching
                cand["graph_intervals"], cand["cull"], cand["batch_trials"] = 0, 0, min(cand["batch_trials"], 1)
                cand["split"] = min(cand["split"], 2)
            rate = trial(cand)
            if rate > best_rate:
                best, best_rate = cand, rate
    result = {"options": best, "trials_per_s": best_rate, "table": table}
    if cache_path:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        cache[sig] = result
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return result
