"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): the library is rebuilt with both sanitizers into a temporary directory and a
child Python process, with the sanitizer runtimes preloaded, runs every oracle entry
point family on small inputs -- plain, learned, paper-schedule and MD chains with
traces, checkpoint and restore, the exchange ratio, energies and observables, the
naive reweighting, its targets, observables, batch means and bootstrap.  Any invalid
access or undefined operation aborts the child."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import sys
sys.path.insert(0, @@ROOT@@)
import numpy as np
import oracle
oracle._LIB_PATH = @@LIB@@
from paper_1908_11118_amd import workloads as W

w = W.small_lj(n_t=2, n_mu=2, n_max=12, mu=(-4.0, -2.5)).replace(sample_every=1)
ch = oracle.Chain(w, n_threads=2, observables=dict(dz=0.25, layer=(0.6, 1.6), dr=0.1, nr=30))
r = ch.run(40, trace=True)
blob = ch.checkpoint()
ch.run(5)
ch.restore(blob)
ch.run(5)
xyz = np.random.default_rng(0).uniform(0.0, 5.0, (6, 3))
ch.energy(xyz)
ch.observables(xyz)
ch.md_forces(xyz)
oracle.swap_lnratio(1.0, -2.0, 0.8, -2.5, -3.0, 4, -1.0, 2)
# learned chain with a seeded network, the paper's schedule with MC and with MD
net = W.mlp_pack(W.mlp_init(3))
oracle.Chain(w, net=net, alpha=0.7, n_threads=2).run(10)
oracle.Chain(W.paper_schedule(w, x0=0.9, mc_cycles=2, sample_every=1), n_threads=2).run(20)
oracle.Chain(W.paper_schedule_md(w, x0=0.8, md_steps=2, sample_every=1), n_threads=2).run(10)
# reweighting
beta, lnz = oracle.state_arrays(w)
e, n, st = r["e"], r["n"], r["state"]
f, logd, ok, _, _ = oracle.mbar_solve(beta, lnz, np.bincount(st, minlength=w.n_states), e, n, tol=1e-9,
                                      n_threads=2)
t = oracle.mbar_targets(beta, lnz, e, n, logd, w.n_max, n_threads=2)
oracle.mbar_observables(beta, lnz, e, n, logd, w.n_max, np.ones((len(e), 3)), n_threads=2)
oracle.batch_means(w.n_states, st, n, 5)
oracle.mbar_bootstrap(beta, lnz, e, n, st, w.n_states, 4, 3, 1, f, beta, lnz, w.n_max, n_threads=2)
oracle.heat_capacity_coverage(beta, t["mean_n"], t["mean_e"], t["mean_e2"], 4.0)
print("sanitized oracle run complete")
'''


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if asan is None or ubsan is None:
        pytest.skip("gcc sanitizer runtimes not installed")
    import oracle
    lib = str(tmp_path / "liboracle_san.so")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-o", lib]
    cmd += [os.path.join(os.path.dirname(oracle.__file__), s) for s in oracle._SOURCES] + ["-lm"]
    subprocess.run(cmd, check=True)
    env = dict(os.environ)
    env["LD_PRELOAD"] = f"{asan}:{ubsan}"
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["OMP_NUM_THREADS"] = "2"
    script = CHILD.replace("@@ROOT@@", repr(ROOT)).replace("@@LIB@@", repr(lib))
    res = subprocess.run([sys.executable, "-c", script], env=env, capture_output=True, text=True, timeout=600)
    assert res.returncode == 0, res.stderr[-4000:]
    assert "sanitized oracle run complete" in res.stdout
    assert "ERROR: AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr, res.stderr[-4000:]
