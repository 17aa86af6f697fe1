"""Benchmark of the REGC sampling hot path on one MI355X.

Workload (1024-replica REGC at a 192-atom slab): 8x8x3 fcc(100) slab, gas box
12^3 sigma, N <= 200, 32 T in [0.5, 2] x 32 mu in [-8, -2] = 1024 replicas, LJ
12-6 truncated and shifted at 2.5 sigma, 50/25/25 displacement/insertion/removal
with K = 201 trials per sweep, exchange every 10 sweeps, FP32 pair terms with FP64
running energies and decisions.  Synthetic inputs (seeded), no dataset.

One step = one exchange interval: 10 sweeps of every walker (the sweep kernel)
followed by the exchange kernel; samples are written every 100 sweeps.  The walkers
are first equilibrated for --burnin sweeps (untimed) so the timed region runs at the
production particle counts.  Metric: GC trial moves per second over all replicas
(every attempted trial counts, rejected or not).

Also reported: the sweep kernel against the FP32 vector roofline (candidate pair
terms x 25 flops / kernel time from HIP events on the context stream), the CPU
oracle's trial rate on the host cores on a bounded sample of the same workload,
and the reweighting of 1024 states x ~10^6 samples.  A last leg measures the
wall time to a target accuracy of <N>(T, mu) with and without the learned insertion
proposal on the 64-replica system (--learned-seconds 0 skips it).  --full-stack adds
the 4096-replica uneven batch with one learned proposal per slab class, per-class
reweighting maps and an FP64 oracle check on a 64-replica subset (off by default:
it takes minutes of GPU and host time).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FLOPS_PER_PAIR = 25.0          # FP32 flops per candidate pair term (FMA = 2, rcp = 1)
PEAK_FP32_TFLOPS = 157.3       # MI355X FP32 vector peak
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "sweep_kernel_f32_1024rep_192slab_traffic.md")
# the sweep kernel's sources and the host code that picks its launch shape
KERNEL_SOURCES = ["sweep.hip", "sweep_dev.h", "regc_dev.h", "philox_dev.h", "api.cpp"]


def measured_traffic():
    """HBM bytes per sweep launch from the committed counter summary, or None when
    the kernel's sources changed since the counters were taken."""
    import hashlib
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    fields = dict(line.split(": ", 1) for line in text.splitlines()
                  if line.startswith(("bytes_per_launch: ", "source_sha256: ")))
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1908_11118_amd", "csrc", f), "rb").read())
    if fields.get("source_sha256", "").strip() != h.hexdigest():
        return None
    return float(fields["bytes_per_launch"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--burnin", type=int, default=3000, help="untimed equilibration sweeps")
    ap.add_argument("--cpu-sweeps", type=int, default=500, help="oracle sweeps timed for cpu_baseline (0: skip)")
    ap.add_argument("--mbar-records", type=int, default=1000, help="records for the reweighting leg (0: skip)")
    ap.add_argument("--production-sweeps", type=int, default=100000,
                    help="sweeps of the production leg: the 1024-replica run sampled every 100 sweeps and "
                         "reweighted over all its samples (0: skip)")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--wpb", type=int, default=0, help="walkers per workgroup (0: the library's choice)")
    ap.add_argument("--split", type=int, default=0, help="waves per walker, 1 or 2 (0: the library's choice)")
    ap.add_argument("--workload", default="c2", choices=["c2", "c3"],
                    help="c2: 1024 replicas at a 192-atom slab (the headline); c3: 4096 replicas in four "
                         "slab classes batched in one launch")
    ap.add_argument("--autotune", action="store_true", help="pick the launch shape with the autotuner first")
    ap.add_argument("--graph", type=int, default=-1, help="graph_intervals (-1: 0 for c2, 10 for c3)")
    ap.add_argument("--learned-seconds", type=float, default=60.0,
                    help="GPU-time cap of the plain and learned runs of the time-to-accuracy leg (0: skip the leg)")
    ap.add_argument("--c3-sweeps", type=int, default=10000,
                    help="sweeps of the 4096-replica uneven batch leg (0: skip)")
    ap.add_argument("--c3-burnin", type=int, default=2000, help="untimed equilibration sweeps of that leg")
    ap.add_argument("--schedule-seconds", type=float, default=0.0,
                    help="GPU-time cap of the runs of that leg with the paper's REGC step (MC and MD forms; "
                         "0: skip them)")
    ap.add_argument("--learned-tau", type=float, default=0.5, help="standard-error target (particles) of that leg")
    ap.add_argument("--learned-alpha", type=float, default=0.9, help="mixture weight of the network branch")
    ap.add_argument("--learned-capture", type=int, default=10000, help="plain sweeps per seed captured for training")
    ap.add_argument("--learned-train-steps", type=int, default=20000, help="Adam steps of the proposal network")
    ap.add_argument("--learned-reference", type=int, default=100000, help="sweeps of the FP64 reference run")
    ap.add_argument("--full-stack", type=int, default=1,
                    help="1: also run the full stack (reduced in length by default): the 4096-replica uneven batch "
                         "with one learned proposal per slab class, per-class reweighting maps with errors and an "
                         "FP64 oracle check on a 64-replica subset; 0: skip")
    ap.add_argument("--fs-capture", type=int, default=200, help="full stack: captured sweeps for training")
    ap.add_argument("--fs-train-steps", type=int, default=2000, help="full stack: Adam steps per class network")
    ap.add_argument("--fs-sweeps", type=int, default=400, help="full stack: production sweeps (sampled every 2)")
    ap.add_argument("--fs-oracle-sweeps", type=int, default=1000, help="full stack: oracle sweeps on the subset")
    ap.add_argument("--fs-boot", type=int, default=20, help="full stack: bootstrap replicates of the error maps")
    ap.add_argument("--fs-tmin", type=float, default=0.88,
                    help="full stack: lowest temperature of the restricted reweighting (below it the states "
                         "on either side of the condensation do not exchange configurations)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU sharding is described in the "
                                   "design notes but not built", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1908_11118_amd import regc
    from paper_1908_11118_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    wl = [W.config2()] if args.workload == "c2" else W.config3_classes()
    w = wl[0]
    n_walkers = sum(x.n_states for x in wl)
    trials_per_sweep_all = sum(x.n_states * x.trials for x in wl)
    sweeps_per_step = w.swap_every
    prec = regc.FP32PAIR if args.precision == "fp32" else regc.FP64
    total_sweeps = args.burnin + (args.warmup + args.steps) * sweeps_per_step
    cap = (total_sweeps // w.sample_every + 2) * n_walkers
    opts = {"walkers_per_block": args.wpb, "split": args.split,
            "graph_intervals": (0 if args.workload == "c2" else 10) if args.graph < 0 else args.graph}
    tuned = None
    if args.autotune:
        from paper_1908_11118_amd import autotune
        print("[bench] autotuning the launch shape", file=sys.stderr, flush=True)
        tuned = autotune.autotune(wl, precision=prec, cache_path=None, verbose=True)
        opts = dict(tuned["options"])
    g = regc.Regc(wl if len(wl) > 1 else w, precision=prec, sample_capacity=cap, **opts)
    print(f"[bench] burn-in {args.burnin} sweeps of {args.workload}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    done = 0
    while done < args.burnin:
        step = min(500, args.burnin - done)
        g.run(step)
        g.sync()
        done += step
        print(f"[bench] burn-in {done}/{args.burnin} sweeps, {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        g.run(sweeps_per_step)
    g.sync()
    st0 = g.stats()["stats"].copy()
    pc0 = g.pair_counts()
    g.timing_enable(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        g.run(sweeps_per_step)
    g.sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    tm = g.timing()
    st1 = g.stats()["stats"]
    pc1 = g.pair_counts()
    trials = args.steps * sweeps_per_step * trials_per_sweep_all
    d = st1 - st0
    assert int(d[:, [0, 2, 4]].sum()) == trials, "trial count mismatch"
    value = trials / elapsed
    cand = pc1[0] - pc0[0]
    useful = pc1[1] - pc0[1]
    ms_kernel = tm["ms_sweep"] / max(tm["n_sweep"], 1)
    flops_launch = FLOPS_PER_PAIR * cand / max(tm["n_sweep"], 1)
    graph = opts.get("graph_intervals", 0) > 0
    achieved = flops_launch / (ms_kernel * 1e-3) / 1e12
    achieved_in = FLOPS_PER_PAIR * useful / max(tm["n_sweep"], 1) / (ms_kernel * 1e-3) / 1e12
    wk = g.walkers(xyz=True)

    acc = {k: float(d[:, 2 * i + 1].sum() / max(d[:, 2 * i].sum(), 1))
           for i, k in enumerate(["displacement", "insertion", "removal"])}
    sw = g.stats()
    swap_rate = float(sw["swap_acc"].sum() / max(sw["swap_att"].sum(), 1))
    result = {
        "metric": "GC trial moves/s (all replicas, 1 GPU); wall-s to <N>(T,mu) at 3 SE, learned vs plain",
        "value": value,
        "unit": "trial moves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == regc.FP32PAIR else "f64",
        "data": "synthetic",
        "config": {"workload": ("REGC 1024 replicas (32 T x 32 mu), 8x8x3 = 192-atom fcc(100) LJ slab, "
                                "gas box 12^3, N <= 200, K = 201 trials/sweep, exchange every 10 sweeps")
                               if args.workload == "c2" else
                               ("REGC 4096 replicas: four slab classes {6,8,10,12}^2 x 3 (108-432 atoms), "
                                "boxes 9-18 x 12, each 32 T x 32 mu, N <= 500, K = 501, one launch per interval"),
                   "replicas": n_walkers, "n_max": w.n_max, "trials_per_sweep": w.trials,
                   "launch": opts,
                   "sweeps_per_step": sweeps_per_step, "burnin_sweeps": args.burnin,
                   "precision": "FP32 pair terms, FP64 energies/decisions/exchange" if prec == regc.FP32PAIR
                   else "FP64", "mean_N": float(wk["n"].mean()), "max_N": int(wk["n"].max())},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS,
                     "basis": "candidate pair terms (gas atoms + slab column block, twice per displacement)",
                     "achieved_in_cutoff": achieved_in, "frac_in_cutoff": achieved_in / PEAK_FP32_TFLOPS,
                     "traffic": measured_traffic() if (args.workload == "c2" and prec == regc.FP32PAIR and not graph)
                     else None,
                     "traffic_unit": "HBM bytes per launch (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, copy-calibrated)",
                     "kernel": "sweep_kernel_f32" if prec == regc.FP32PAIR else "sweep_kernel_f64",
                     "kernel_ms_avg": ms_kernel, "launches": tm["n_sweep"],
                     "timed_unit": "graph replay (sweeps + exchange)" if graph else "sweep-kernel launch",
                     "candidate_pairs_per_launch": cand / max(tm["n_sweep"], 1),
                     "flops_per_pair": FLOPS_PER_PAIR,
                     "useful_pair_fraction": useful / max(cand, 1)},
        "acceptance": acc,
        "swap_acceptance": swap_rate,
        "kernel_share": tm["ms_sweep"] / (elapsed * 1e3),
    }

    if tuned is not None:
        result["autotune"] = {"chosen": tuned["options"], "table": tuned["table"]}
    # ---- CPU baseline: the FP64 oracle on the host cores, same configurations ----
    if args.cpu_sweeps > 0 and args.workload == "c2":
        import oracle
        oracle.build(force=False)
        threads = oracle.default_threads()
        ch = oracle.Chain(w.replace(sample_every=0), n_threads=threads)
        ch.set_walkers(wk["n"], wk["xyz"], label=wk["label"])
        ch.sweep[0] = g.sweep
        print(f"[bench] cpu baseline: {args.cpu_sweeps} oracle sweeps on {threads} threads",
              file=sys.stderr, flush=True)
        c0 = time.perf_counter()
        ch.run(args.cpu_sweeps)
        csec = time.perf_counter() - c0
        ctrials = args.cpu_sweeps * w.n_states * w.trials
        result["cpu_baseline"] = {"value": ctrials / csec, "unit": "trial moves/s", "cores": threads,
                                  "kind": "oracle",
                                  "sample": f"{args.cpu_sweeps} sweeps x 1024 replicas x 201 trials of the same "
                                            f"workload from the GPU's equilibrated configurations (FP64), "
                                            f"{csec:.1f} s"}

    # ---- production leg: the configuration the metric is quoted on, end to end ----
    if args.production_sweeps > 0 and args.workload == "c2":
        result["production"] = production_leg(args, w, wk, prec)

    # ---- reweighting leg: 1024 states x mbar-records records ----
    if args.mbar_records > 0 and args.workload == "c2":
        g.close()
        wm = w.replace(sample_every=1)
        gm = regc.Regc(wm, precision=prec, sample_capacity=args.mbar_records * w.n_states,
                       walkers_per_block=args.wpb)
        gm.set_walkers(wk["n"], wk["xyz"], label=wk["label"])
        # structural observables with every record: axial density in 0.12-sigma bins and
        # the lateral pair distribution of the first adsorbed layer (0.6 <= z < 1.6)
        gm.set_observables(0.12, (0.6, 1.6), 0.05, 120)
        gm.track_minima(True)
        print(f"[bench] reweighting leg: collecting {args.mbar_records} records", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t_rec = time.perf_counter()
        gm.run(args.mbar_records)
        gm.sync()
        t_rec = time.perf_counter() - t_rec
        mb = regc.Mbar(w.t, w.mu, w.n_max)
        mb.load_run(gm, 0, 0)
        ns = args.mbar_records * w.n_states
        f, conv, iters, delta = mb.solve(tol=1e-8, max_iter=2000, allow_noconv=True)
        ms, nit = mb.timing()
        tr = mb.targets(W.linear_grid(0.5, 2.0, 64), W.linear_grid(-8.0, -2.0, 64))
        per_iter = ms / max(nit, 1)
        L = len(w.t)
        tt_obs = W.linear_grid(0.5, 2.0, 16)
        t_obs = time.perf_counter()
        mean_o, cond_o = mb.observables(tt_obs, W.linear_grid(-8.0, -2.0, 64), gm.n_obs)
        t_obs = time.perf_counter() - t_obs
        result["observables"] = {"n_obs": gm.n_obs, "bins": f"{gm.n_obs - 121} axial (0.12) + 120 lateral (0.05, layer 0.6-1.6) + 1",
                                 "recording_ms_per_record": 1e3 * t_rec / args.mbar_records,
                                 "reweight_targets": "16 T x 64 mu", "reweight_s": t_obs,
                                 "fp64_fma_per_s": 16 * ns * gm.n_obs / t_obs}
        # aiAT@REGC phase map (lowest sampled energy per N) against the reweighted one
        e_min, _ = gm.minima(0)
        tmu = W.linear_grid(-8.0, -2.0, 64)
        ai = regc.aiat_phase(e_min, tmu)
        mb_phase = np.asarray(tr["phase"]).reshape(64, 64)
        agree = mb_phase == ai[None, :]
        low = mb_phase <= w.n_max // 4
        result["aiat_vs_mbar"] = {"grid": "64 T x 64 mu", "agree_fraction": float(agree.mean()),
                                  "agree_fraction_where_mbar_N_le_nmax_4": float(agree[low].mean()) if low.any()
                                  else None,
                                  "aiat_phases": int(len(set(ai.tolist()))),
                                  "mbar_phases": int(len(set(mb_phase.ravel().tolist())))}
        result["mbar"] = {"states": w.n_states, "samples": ns, "iterations": nit, "converged": bool(conv),
                          "max_delta_f": delta, "ms_per_iteration": per_iter,
                          "fp64_exp_per_s": L * ns / (per_iter * 1e-3),
                          "sample_stream_GBps": 8.0 * ns / (per_iter * 1e-3) / 1e9,
                          "target_grid": "64 x 64", "phases_found": int(len(set(tr["phase"].tolist())))}
        # consistency at the sampled states: reweighted <N> against the direct per-state
        # means, for the solve over all states and for the solve over T >= 0.88 only (the
        # low-T rows do not exchange configurations across the condensation)
        smp = gm.samples()
        S = w.n_states
        m_dir, se_dir = regc.batch_means(smp["state"], smp["n"], S)
        at = mb.targets(w.t, w.mu)["mean_n"]
        l0 = int(np.searchsorted(w.t, 0.88))
        keep = smp["state"] // len(w.mu) >= l0
        mh = regc.Mbar(w.t[l0:], w.mu, w.n_max)
        mh.set_samples(smp["e"][keep], smp["n"][keep], smp["state"][keep] - l0 * len(w.mu))
        mh.solve(tol=1e-8, max_iter=2000, allow_noconv=True)
        ah = mh.targets(w.t[l0:], w.mu)["mean_n"]
        mh.close()
        hi = np.arange(S) >= l0 * len(w.mu)
        se_f = np.maximum(se_dir, 0.02)
        z_all = (at - m_dir) / se_f
        z_hi = (ah - m_dir[hi]) / se_f[hi]
        if args.cpu_sweeps > 0:
            # the oracle's naive reweighting iteration (every state x every sample) on the host
            # cores, timed on the first 1e5 samples and scaled to the full set
            import oracle
            oracle.build(force=False)
            sub = min(ns, 100000)
            beta_s, lnz_s = oracle.state_arrays(w)
            om = np.bincount(smp["state"][:sub], minlength=S)
            t_c = time.perf_counter()
            oracle.mbar_iterate(beta_s, lnz_s, om, smp["e"][:sub], smp["n"][:sub], np.zeros(S))
            t_c = time.perf_counter() - t_c
            result["mbar"]["cpu_baseline"] = {
                "kind": "oracle", "cores": oracle.default_threads(),
                "sample": f"one naive iteration over {S} states x the first {sub} samples, {t_c:.2f} s",
                "seconds_per_iteration_full_set": t_c * ns / sub,
                "gpu_over_cpu_per_iteration": (t_c * ns / sub) / (per_iter * 1e-3)}
        result["mbar"]["consistency_at_sampled_states_t_ge_0.88"] = {
            "states": int(hi.sum()),
            "all_state_solve": {"mean_z": float(z_all[hi].mean()), "frac_abs_z_gt_3": float(np.mean(np.abs(z_all[hi]) > 3))},
            "restricted_solve": {"mean_z": float(z_hi.mean()), "frac_abs_z_gt_3": float(np.mean(np.abs(z_hi) > 3))}}
        mb.close()
        gm.close()
    if args.c3_sweeps > 0 and args.workload == "c2":
        g.close()
        result["c3"] = c3_leg(args, prec)
    if args.learned_seconds > 0:
        result["learned"] = learned_leg(args)
    if args.full_stack:
        result["full_stack"] = full_stack_leg(args)
    print(json.dumps(result))


def production_leg(args, w, wk, prec):
    """The 1024-replica run at its stated length: production_sweeps sweeps from the
    benchmark's equilibrated walkers, samples every 100 sweeps (1.024e6 for 1e5
    sweeps), graph-replayed exchange intervals; then the reweighting of every sample
    into <N>, the coverage and the phase map on a 64 x 64 grid."""
    import numpy as np
    import torch

    from paper_1908_11118_amd import regc
    from paper_1908_11118_amd import workloads as W

    say = lambda m: print(m, file=sys.stderr, flush=True)
    n_rec = args.production_sweeps // w.sample_every
    out = {"sweeps": args.production_sweeps, "sample_every": w.sample_every, "records": n_rec}
    with regc.Regc(w, precision=prec, sample_capacity=max(n_rec, 1) * w.n_states, graph_intervals=10) as g:
        g.set_walkers(wk["n"], wk["xyz"], label=wk["label"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done, chunk = 0, 10000
        while done < args.production_sweeps:
            k = min(chunk, args.production_sweeps - done)
            g.run(k)
            g.sync()
            done += k
            say(f"[production] {done}/{args.production_sweeps} sweeps, {time.perf_counter() - t0:.1f} s")
        t_run = time.perf_counter() - t0
        out["seconds"] = t_run
        out["trial_moves_per_s"] = args.production_sweeps * w.n_states * w.trials / t_run
        mb = regc.Mbar(w.t, w.mu, w.n_max)
        skip = n_rec // 10
        mb.load_run(g, 0, skip)
        t0 = time.perf_counter()
        f, conv, iters, delta = mb.solve(tol=1e-8, max_iter=3000, allow_noconv=True)
        t_mb = time.perf_counter() - t0
        # estimates with errors on a 64 x 64 grid: coverage of the 8 x 8 hollow sites of
        # the slab's top layer and heat capacity, bootstrap SEs over 100 replicates
        tg = W.linear_grid(0.5, 2.0, 64), W.linear_grid(-8.0, -2.0, 64)
        t0 = time.perf_counter()
        rw = mb.reweight(*tg, tol=1e-8, max_iter=3000, n_batches=20, n_boot=100, n_sites=64.0, allow_noconv=True)
        t_rw = time.perf_counter() - t0
        mb.close()
    out["reweighting"] = {"samples": (n_rec - skip) * w.n_states, "iterations": iters, "converged": bool(conv),
                          "seconds": t_mb, "target_grid": "64 T x 64 mu",
                          "phases": int(len(set(rw["phase"].tolist()))),
                          "coverage_range": [float(rw["coverage"].min()), float(rw["coverage"].max())],
                          "coverage_se_max": float(np.nanmax(rw["se_coverage"])),
                          "coverage_se_median": float(np.nanmedian(rw["se_coverage"])),
                          "heat_capacity_max": float(rw["heat_cap"].max()),
                          "heat_capacity_se_median": float(np.nanmedian(rw["se_heat_cap"])),
                          "mean_n_se_max": float(np.nanmax(rw["se_n"])),
                          "sampled_states_se_max": float(np.nanmax(rw["se_state_n"])),
                          "errors": "bootstrap over 100 replicates of blocks of records (targets), batch means of "
                                    "20 batches (sampled states)",
                          "estimates_with_errors_seconds": t_rw, "estimates_converged": bool(rw["converged"])}
    say(f"[production] {out}")
    return out


def c3_leg(args, prec):
    """The 4096-replica uneven batch: four slab classes {6,8,10,12}^2 x 3 (108-432
    atoms), boxes 1.5 n x 1.5 n x 12, each class a 32 T x 32 mu grid, N <= 500, K = 501,
    exchange every 10 sweeps, ten exchange intervals (100 sweeps) per graph replay; c3_sweeps timed sweeps
    after c3_burnin untimed ones.  Throughput and the sweep kernel against the FP32
    roofline on both the candidate and the in-cutoff basis."""
    import torch

    from paper_1908_11118_amd import regc
    from paper_1908_11118_amd import workloads as W

    say = lambda m: print(m, file=sys.stderr, flush=True)
    wl = W.config3_classes()
    n_w = sum(x.n_states for x in wl)
    per_sweep = sum(x.n_states * x.trials for x in wl)
    recs = (args.c3_burnin + args.c3_sweeps) // wl[0].sample_every + 2
    out = {"workload": "REGC 4096 replicas: four slab classes {6,8,10,12}^2 x 3 (108-432 atoms), boxes 9-18 x 12, "
                       "each 32 T x 32 mu, N <= 500, K = 501, exchange every 10 sweeps, one graph replay per ten "
                       "exchange intervals (100 sweeps)",
           "sweeps": args.c3_sweeps, "burnin_sweeps": args.c3_burnin}
    with regc.Regc(wl, precision=prec, sample_capacity=recs * n_w, graph_intervals=10) as g:
        t0 = time.perf_counter()
        done = 0
        while done < args.c3_burnin:
            k = min(1000, args.c3_burnin - done)
            g.run(k)
            g.sync()
            done += k
            say(f"[c3] burn-in {done}/{args.c3_burnin} sweeps, {time.perf_counter() - t0:.1f} s")
        st0 = g.stats()["stats"].copy()
        pc0 = g.pair_counts()
        g.timing_enable(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = 0
        while done < args.c3_sweeps:
            k = min(2000, args.c3_sweeps - done)
            g.run(k)
            g.sync()
            done += k
            say(f"[c3] {done}/{args.c3_sweeps} sweeps, {time.perf_counter() - t0:.1f} s")
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        tm = g.timing()
        d = g.stats()["stats"] - st0
        pc1 = g.pair_counts()
        wk = g.walkers()
    trials = int(d[:, [0, 2, 4]].sum())
    assert trials == args.c3_sweeps * per_sweep, "trial count mismatch"
    cand, useful = pc1[0] - pc0[0], pc1[1] - pc0[1]
    ms = tm["ms_sweep"]
    achieved = FLOPS_PER_PAIR * cand / (ms * 1e-3) / 1e12
    achieved_in = FLOPS_PER_PAIR * useful / (ms * 1e-3) / 1e12
    out.update({"value": trials / elapsed, "unit": "trial moves/s", "seconds": elapsed,
                "mean_N": float(wk["n"].mean()), "max_N": int(wk["n"].max()),
                "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                             "frac": achieved / PEAK_FP32_TFLOPS,
                             "basis": "candidate pair terms (gas atoms + slab column block, twice per displacement)",
                             "achieved_in_cutoff": achieved_in, "frac_in_cutoff": achieved_in / PEAK_FP32_TFLOPS,
                             "traffic": None,
                             "timed_unit": "graph replay (10 exchange intervals: 100 sweeps + 10 exchanges), HIP "
                                           "events on the context stream",
                             "replays": tm["n_sweep"], "ms_per_replay": ms / max(tm["n_sweep"], 1),
                             "candidate_pairs_per_replay": cand / max(tm["n_sweep"], 1),
                             "useful_pair_fraction": useful / max(cand, 1), "flops_per_pair": FLOPS_PER_PAIR}})
    say(f"[c3] {out['value']:.3g} trial moves/s")
    return out


def learned_leg(args):
    """Time to accuracy of <N>(T, mu) with and without the learned insertion
    proposal on the 64-replica system (4x4x2 slab, box 6x6x8, N <= 40): training
    data from plain runs (seeds 1, 2), training on the GPU, a long FP64 reference
    run (seed 4), then both forms from the same equilibrated state (seed 3)."""
    import numpy as np
    import torch

    from paper_1908_11118_amd import proposal as P
    from paper_1908_11118_amd import regc
    from paper_1908_11118_amd import workloads as W

    say = lambda m: print(m, file=sys.stderr, flush=True)
    w = W.config1()
    out = {"workload": "64 replicas (8 T x 8 mu), 4x4x2 = 32-atom slab, box 6x6x8, N <= 40, K = 41",
           "alpha": args.learned_alpha, "tau": args.learned_tau, "frac_within_3se": 0.98, "max_chi2": 1.3,
           "precision": "FP32 pair terms; network bf16 on MFMA"}
    t = time.perf_counter()
    vox, n = P.capture_dataset(w, seeds=(1, 2), burnin=2000, sweeps=args.learned_capture)
    torch.cuda.synchronize()
    out["training_examples"] = int(vox.shape[0])
    out["capture_s"] = time.perf_counter() - t
    say(f"[learned] captured {vox.shape[0]} configurations in {out['capture_s']:.1f} s")
    t = time.perf_counter()
    net = P.train(vox, n, steps=args.learned_train_steps, batch=256, lr=1e-3)
    torch.cuda.synchronize()
    out["train_s"] = time.perf_counter() - t
    out["train_steps"] = args.learned_train_steps
    # cross-entropy on 4096 random training examples (in-sample), against the uniform proposal's ln 4096
    rng = np.random.default_rng(5)
    vh = vox[:min(200000, int(vox.shape[0]))].cpu().numpy().view(np.uint16)
    nh = n[:min(200000, int(n.shape[0]))].cpu().numpy()
    sel = rng.choice(np.nonzero(nh > 0)[0], 4096, replace=False)
    excl = rng.integers(0, nh[sel]).astype(np.int32)
    target = vh[sel, excl].astype(np.int32)
    loss, _ = net.loss_grads(vh[sel], nh[sel], excl, target)
    out["loss_after"] = loss
    out["loss_uniform"] = float(np.log(4096.0))
    del vox, n
    say(f"[learned] trained in {out['train_s']:.1f} s, loss {loss:.3f} (uniform {np.log(4096.0):.3f})")
    t = time.perf_counter()
    ref_m, ref_se = P.reference(w, sweeps=args.learned_reference)
    out["reference"] = {"sweeps": args.learned_reference, "precision": "FP64", "seconds": time.perf_counter() - t,
                        "max_se": float(ref_se.max())}
    blob = P.equilibrated_state(w)
    # both forms run until the target is met or --learned-seconds of GPU time are spent
    # (no sweep cap: the plain form's worst state, at the condensation step, has a noisy
    # error estimate and can need more than 2e5 sweeps)
    plain = P.time_to_accuracy(w, blob, ref_m, ref_se, tau=args.learned_tau, max_seconds=args.learned_seconds,
                               max_sweeps=10 ** 8, log=say)
    say(f"[learned] plain: reached={plain['reached']} t={plain['t_acc_s']:.2f} s sweeps={plain['sweeps']}")
    learned = P.time_to_accuracy(w, blob, ref_m, ref_se, net=net, alpha=args.learned_alpha, tau=args.learned_tau,
                                 max_seconds=args.learned_seconds, max_sweeps=10 ** 8, log=say)
    say(f"[learned] learned: reached={learned['reached']} t={learned['t_acc_s']:.2f} s sweeps={learned['sweeps']}")
    net.close()
    keep = ("reached", "t_acc_s", "sweeps", "max_se", "frac_within", "chi2", "ins_acc", "ms_per_sweep")
    out["plain"] = {k: plain[k] for k in keep}
    if args.schedule_seconds > 0:
        # the paper's REGC step (x0 = 0.99, 10 MC cycles of N displacements) from the same state
        wp = W.paper_schedule(w, x0=0.99, mc_cycles=10, sample_every=1)
        paper = P.time_to_accuracy(wp, blob, ref_m, ref_se, tau=args.learned_tau, chunk=50,
                                   max_seconds=args.schedule_seconds, log=say)
        say(f"[learned] paper schedule: reached={paper['reached']} t={paper['t_acc_s']:.2f} s "
            f"steps={paper['sweeps']}")
        # the same step with molecular dynamics as the canonical part (REGCMD)
        wmd = W.paper_schedule_md(w, x0=0.99, md_steps=10, md_dt=0.005, md_tau=0.1, sample_every=1)
        pmd = P.time_to_accuracy(wmd, blob, ref_m, ref_se, tau=args.learned_tau, chunk=50,
                                 max_seconds=args.schedule_seconds, log=say)
        say(f"[learned] paper schedule, MD: reached={pmd['reached']} t={pmd['t_acc_s']:.2f} s steps={pmd['sweeps']}")
        out["paper_schedule_md"] = {k: pmd[k] for k in keep}
        out["paper_schedule_md"]["steps"] = out["paper_schedule_md"].pop("sweeps")
        out["paper_schedule_md"]["ms_per_step"] = out["paper_schedule_md"].pop("ms_per_sweep")
        out["paper_schedule_md"].update({"x0": 0.99, "md_steps": 10, "md_dt": 0.005, "md_tau": 0.1})
        out["paper_schedule"] = {k: paper[k] for k in keep}
        out["paper_schedule"]["steps"] = out["paper_schedule"].pop("sweeps")
        out["paper_schedule"]["ms_per_step"] = out["paper_schedule"].pop("ms_per_sweep")
        out["paper_schedule"]["x0"], out["paper_schedule"]["mc_cycles"] = 0.99, 10
        out["efficiency_ratio_paper_schedule_over_plain"] = P.efficiency_ratio(plain, paper)
        out["efficiency_ratio_paper_schedule_md_over_plain"] = P.efficiency_ratio(plain, pmd)
        if plain["reached"] and paper["reached"]:
            out["paper_schedule"]["t_acc_ratio_plain_over_paper"] = plain["t_acc_s"] / paper["t_acc_s"]
    out["learned"] = {k: learned[k] for k in keep}
    out["learned"]["proposal"] = learned.get("proposal")
    out["efficiency_ratio_learned_over_plain"] = P.efficiency_ratio(plain, learned)
    if plain["reached"] and learned["reached"]:
        out["speedup_t_acc"] = plain["t_acc_s"] / learned["t_acc_s"]
    elif plain["reached"]:
        out["speedup_t_acc"] = f"< {plain['t_acc_s'] / learned['t_acc_s']:.4f} (learned not reached in the cap)"
    return out


def oracle_heat_capacity(w, r):
    """The oracle's heat capacity at each sampled state of an oracle run r: its own
    reweighting of that state's samples alone (the plain sample moments)."""
    import numpy as np

    import oracle
    beta, lnz = oracle.state_arrays(w)
    out = np.zeros(w.n_states)
    for k in range(w.n_states):
        sel = r["state"] == k
        e, n = r["e"][sel], r["n"][sel]
        _, logd, _, _, _ = oracle.mbar_solve(beta[k:k + 1], lnz[k:k + 1], [int(sel.sum())], e, n, tol=1e-12)
        t = oracle.mbar_targets(beta[k:k + 1], lnz[k:k + 1], e, n, logd, w.n_max)
        out[k] = oracle.heat_capacity_coverage(beta[k:k + 1], t["mean_n"], t["mean_e"], t["mean_e2"], 1.0)[0][0]
    return out


def full_stack_leg(args):
    """4096 uneven replicas (four slab classes 6x6 .. 12x12 x 3, N <= 500) with one
    learned insertion proposal per class fused into the sweep, FP32 pairs; the
    reweighting of each class (1024 states) into <N>, coverage and heat-capacity
    maps; the maps checked against the FP64 oracle run as its own REGC on an 8 x 8
    sub-grid of the 6x6 class, started from the GPU's configurations."""
    import numpy as np
    import torch

    import oracle
    from paper_1908_11118_amd import proposal as P
    from paper_1908_11118_amd import regc
    from paper_1908_11118_amd import workloads as W

    say = lambda m: print(m, file=sys.stderr, flush=True)
    classes = W.config3_classes()
    out = {"workload": "4 slab classes {6,8,10,12}^2 x 3, box 1.5n x 1.5n x 12, N <= 500, 4 x 32 x 32 replicas",
           "alpha": args.learned_alpha,
           "reduced": {"production_sweeps": args.fs_sweeps, "stated_sweeps": 100000,
                       "samples_per_class": (args.fs_sweeps // 2 - args.fs_sweeps // 20) * 1024,
                       "stated_samples": 4000000, "oracle_sweeps": args.fs_oracle_sweeps,
                       "reason": "the learned sweep runs ~40x slower than the plain one at this size, so the "
                                 "stated 1e5 sweeps would take about two hours"}}
    t = time.perf_counter()
    data, blob = P.capture_batch(classes, burnin=2000, sweeps=args.fs_capture)
    torch.cuda.synchronize()
    out["capture"] = {"sweeps": args.fs_capture, "examples_per_class": int(data[0][0].shape[0]),
                      "seconds": time.perf_counter() - t}
    say(f"[full stack] captured {args.fs_capture} sweeps in {out['capture']['seconds']:.1f} s")
    nets = []
    t = time.perf_counter()
    for c, (vox, n) in enumerate(data):
        nets.append(P.train(vox, n, steps=args.fs_train_steps, batch=256, lr=1e-3, seed=100 + 17 * c))
    torch.cuda.synchronize()
    out["train"] = {"steps_per_class": args.fs_train_steps, "seconds": time.perf_counter() - t}
    del data
    say(f"[full stack] trained {len(nets)} networks in {out['train']['seconds']:.1f} s")

    wl = [w.replace(sample_every=2) for w in classes]
    n_rec = args.fs_sweeps // 2
    Wa = sum(w.n_states for w in wl)
    rates = {}
    with regc.Regc(wl, precision=regc.FP32PAIR, sample_capacity=n_rec * Wa, graph_intervals=10) as g:
        for mode in ("plain", "learned"):
            g.restore(blob)
            for c, net in enumerate(nets):
                g.set_proposal(net if mode == "learned" else None, args.learned_alpha, cls=c)
            g.run(20)
            g.sync()
            t0 = time.perf_counter()
            g.run(40)
            g.sync()
            dt = time.perf_counter() - t0
            rates[mode] = 40 * sum(w.n_states * w.trials for w in wl) / dt
            say(f"[full stack] {mode}: {rates[mode]:.3g} trial moves/s")
        g.clear_samples()
        t0 = time.perf_counter()
        g.run(args.fs_sweeps)
        g.sync()
        t_prod = time.perf_counter() - t0
        ps = g.proposal_stats()
        smp = g.samples()
        wk = g.walkers()
        offs, cnts = g.offsets, g.counts
        out["rates"] = {"plain_trial_moves_per_s": rates["plain"], "learned_trial_moves_per_s": rates["learned"],
                        "production_sweeps": args.fs_sweeps, "production_s": t_prod, "proposal": ps}
        # per-class reweighting over the class's own states: all states, and the states with
        # T >= fs_tmin only (the low-T rows cannot exchange configurations across the
        # condensation, so their samples are not all from equilibrium and bias a joint solve)
        skip = n_rec // 10
        maps, maps_hi = [], []
        for c, w in enumerate(wl):
            n_sites = float(int(round(w.lx / 1.5)) ** 2)       # hollow sites of the top layer
            mb = regc.Mbar(w.t, w.mu, w.n_max)
            mb.load_run(g, c, skip)
            t0 = time.perf_counter()
            f, conv, iters, delta = mb.solve(tol=1e-8, max_iter=3000, allow_noconv=True)
            dt = time.perf_counter() - t0
            tr = mb.reweight(w.t, w.mu, tol=1e-8, max_iter=3000, n_boot=args.fs_boot, n_sites=n_sites,
                             allow_noconv=True)
            mb.close()
            o, cn = offs[c], cnts[c]
            E = smp["e"].reshape(-1, Wa)[skip:, o:o + cn].ravel()
            Nn = smp["n"].reshape(-1, Wa)[skip:, o:o + cn].ravel()
            St = smp["state"].reshape(-1, Wa)[skip:, o:o + cn].ravel()
            l0 = int(np.searchsorted(w.t, args.fs_tmin))
            keep = St // len(w.mu) >= l0
            mh = regc.Mbar(w.t[l0:], w.mu, w.n_max)
            mh.set_samples(E[keep], Nn[keep], St[keep] - l0 * len(w.mu))
            _, conv_h, it_h, _ = mh.solve(tol=1e-8, max_iter=3000, allow_noconv=True)
            trh = mh.reweight(w.t[l0:], w.mu, tol=1e-8, max_iter=3000, n_boot=args.fs_boot, n_sites=n_sites,
                              allow_noconv=True)
            mh.close()
            cov, heat = tr["coverage"], tr["heat_cap"]
            maps.append(tr)
            maps_hi.append((l0, trh))
            out.setdefault("reweighting", []).append(
                {"class": w.name, "samples": int(len(E)), "iterations": iters, "converged": bool(conv),
                 "seconds": dt, "coverage_range": [float(cov.min()), float(cov.max())],
                 "coverage_se_median": float(np.nanmedian(tr["se_coverage"])),
                 "heat_capacity_max": float(heat.max()),
                 "heat_capacity_se_median": float(np.nanmedian(tr["se_heat_cap"])),
                 "phases": int(len(set(tr["phase"].tolist()))),
                 "restricted_t_min": float(w.t[l0]), "restricted_iterations": it_h,
                 "restricted_converged": bool(conv_h)})
            say(f"[full stack] class {c}: reweighting {iters} iterations, {dt:.2f} s")
    for net in nets:
        net.close()

    # FP64 oracle on the 8 x 8 sub-grid (every fourth T and mu) of the 6x6 class, run as
    # its own REGC from the GPU's configurations of those states
    w0 = wl[0]
    sub_t, sub_mu = w0.t[::4], w0.mu[::4]
    ws = w0.replace(t=sub_t, mu=sub_mu, sample_every=1, seed=5)
    lab = wk["label"][offs[0]:offs[0] + cnts[0]]
    li, mi = lab // len(w0.mu), lab % len(w0.mu)
    pick = np.nonzero((li % 4 == 0) & (mi % 4 == 0))[0]
    sub_label = (li[pick] // 4) * len(sub_mu) + mi[pick] // 4
    oracle.build(force=False)
    ch = oracle.Chain(ws, n_threads=oracle.default_threads())
    ch.set_walkers(wk["n"][offs[0] + pick], wk["xyz"][offs[0] + pick], label=sub_label)
    t0 = time.perf_counter()
    ch.run(200)
    r = ch.run(args.fs_oracle_sweeps)
    t_or = time.perf_counter() - t0
    S = ws.n_states
    m_or, se_or = oracle.batch_means(S, r["state"], r["n"], 20)
    sm_n = smp["n"].reshape(-1, Wa)[skip:, offs[0]:offs[0] + cnts[0]].ravel()
    sm_s = smp["state"].reshape(-1, Wa)[skip:, offs[0]:offs[0] + cnts[0]].ravel()
    m_gpu, se_gpu = regc.batch_means(sm_s, sm_n, cnts[0])
    sub_states = np.array([(4 * a) * len(w0.mu) + 4 * b for a in range(len(sub_t)) for b in range(len(sub_mu))])
    se_c = np.maximum(np.sqrt(se_or ** 2 + se_gpu[sub_states] ** 2), 0.02)     # floor: states pinned at the cap
    hi = np.repeat(sub_t >= args.fs_tmin, len(sub_mu))

    def compare(est, sel):
        z = (est[sel] - m_or[sel]) / se_c[sel]
        return {"states": int(sel.sum()), "frac_within_3se": float(np.mean(np.abs(z) <= 3.0)),
                "chi2_per_state": float(np.mean(z ** 2)), "max_abs_dn": float(np.max(np.abs(est[sel] - m_or[sel])))}

    l0, trh = maps_hi[0]
    mbar_all = maps[0]["mean_n"][sub_states]
    mbar_hi = np.full(len(sub_states), np.nan)
    mbar_hi[hi] = trh["mean_n"][sub_states[hi] - l0 * len(w0.mu)]
    heat_or = oracle_heat_capacity(ws, r)
    heat_hi = np.full(len(sub_states), np.nan)
    heat_hi[hi] = trh["heat_cap"][sub_states[hi] - l0 * len(w0.mu)]
    out["oracle_subset"] = {
        "grid": "8 x 8 (every fourth T and mu of the 6x6 class), its own REGC from the GPU's configurations",
        "sweeps": args.fs_oracle_sweeps, "seconds": t_or, "threads": oracle.default_threads(),
        "gpu_direct_means_all_states": compare(m_gpu[sub_states], np.ones(len(sub_states), bool)),
        "reweighted_all_states_solve_at_t_ge_tmin": compare(mbar_all, hi),
        "reweighted_restricted_solve_at_t_ge_tmin": compare(mbar_hi, hi),
        "heat_capacity_restricted_median_rel_diff": float(np.median(np.abs(heat_hi[hi] - heat_or[hi]) /
                                                                    np.maximum(np.abs(heat_or[hi]), 1e-9))),
        "t_min": args.fs_tmin}
    out["oracle_subset_states"] = {"t": np.repeat(sub_t, len(sub_mu)).tolist(), "mu": np.tile(sub_mu, len(sub_t)).tolist(),
                                   "oracle_mean_n": m_or.tolist(), "oracle_se": se_or.tolist(),
                                   "gpu_direct_mean_n": m_gpu[sub_states].tolist(),
                                   "gpu_se": se_gpu[sub_states].tolist(), "reweighted_all": mbar_all.tolist(),
                                   "reweighted_restricted": [None if np.isnan(x) else float(x) for x in mbar_hi],
                                   "heat_capacity_oracle": heat_or.tolist(),
                                   "heat_capacity_restricted": [None if np.isnan(x) else float(x) for x in heat_hi]}
    say(f"[full stack] oracle subset: {out['oracle_subset']}")
    return out


if __name__ == "__main__":
    main()
