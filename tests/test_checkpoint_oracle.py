"""Checkpoint of the oracle's chain: a run killed between sweeps continues from its
last checkpoint exactly as the uninterrupted run does (every random number is keyed by
(trial, sweep, walker), so the state between sweeps is the whole state).

The child process below runs the oracle in chunks of sweeps and writes a checkpoint
after each chunk (write, then atomic rename); the test kills it with SIGKILL once a
checkpoint exists, restores that checkpoint in a fresh chain and runs to the end."""
import os
import subprocess
import sys
import time

import numpy as np
import pytest

import oracle
from paper_1908_11118_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import os, sys
sys.path.insert(0, {root!r})
import oracle
from paper_1908_11118_amd import workloads as W
w = W.small_lj(n_t=2, n_mu=3, n_max=14, n_sweeps=0).replace(seed=11, swap_every=5, sample_every=2)
ch = oracle.Chain(w, n_threads=1)
path = {path!r}
while True:
    ch.run(7)
    blob = ch.checkpoint()
    with open(path + ".tmp", "wb") as f:
        f.write(blob)
    os.replace(path + ".tmp", path)
    print(int(ch.sweep[0]), flush=True)
"""


def _workload():
    return W.small_lj(n_t=2, n_mu=3, n_max=14, n_sweeps=0).replace(seed=11, swap_every=5, sample_every=2)


def _state(ch):
    xyz = [ch.xyz[w, : ch.n[w]].copy() for w in range(ch.S)]
    return dict(n=ch.n.copy(), e=ch.e.copy(), label=ch.label.copy(), wos=ch.wos.copy(), xyz=xyz,
                stats=ch.stats.copy(), att=ch.swap_att.copy(), acc=ch.swap_acc.copy(), sweep=int(ch.sweep[0]))


def _same(a, b):
    for k in ("n", "label", "wos", "stats", "att", "acc"):
        assert np.array_equal(a[k], b[k]), k
    assert a["sweep"] == b["sweep"]
    assert np.array_equal(a["e"], b["e"])          # the same FP64 operations in the same order
    for x, y in zip(a["xyz"], b["xyz"]):
        assert np.array_equal(x, y)


def test_checkpoint_round_trip_in_process():
    w = _workload()
    a = oracle.Chain(w, n_threads=1)
    a.run(23)
    blob = a.checkpoint()
    b = oracle.Chain(w, n_threads=1)
    b.restore(blob)
    _same(_state(a), _state(b))
    ra, rb = a.run(31), b.run(31)
    _same(_state(a), _state(b))
    for k in ("e", "n", "state"):
        assert np.array_equal(ra[k], rb[k])


def test_restore_rejects_a_foreign_or_corrupt_blob():
    w = _workload()
    a = oracle.Chain(w, n_threads=1)
    a.run(5)
    blob = bytearray(a.checkpoint())
    other = oracle.Chain(w.replace(seed=12), n_threads=1)
    with pytest.raises(ValueError):
        other.restore(bytes(blob))                 # another seed
    b = oracle.Chain(w, n_threads=1)
    before = _state(b)
    bad = bytearray(blob)
    bad[40:44] = (10 ** 6).to_bytes(4, "little", signed=True)   # N of walker 0 beyond n_max
    with pytest.raises(ValueError):
        b.restore(bytes(bad))
    _same(before, _state(b))                       # nothing changed
    with pytest.raises(ValueError):
        b.restore(bytes(blob[:-8]))                # truncated


def test_killed_run_continues_from_its_last_checkpoint(tmp_path):
    path = str(tmp_path / "regc.ckpt")
    proc = subprocess.Popen([sys.executable, "-c", CHILD.format(root=ROOT, path=path)],
                            stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)
    try:
        deadline = time.time() + 120
        done = 0
        while done < 21 and time.time() < deadline:   # at least three checkpoints written
            line = proc.stdout.readline()
            if not line:
                break
            done = int(line)
        assert done >= 21, f"child made no progress: {proc.stderr.read() if proc.poll() is not None else ''}"
    finally:
        proc.kill()                                   # SIGKILL: no chance to clean up
        proc.wait()
    assert proc.returncode == -9
    with open(path, "rb") as f:
        blob = f.read()
    total = 70
    resumed = oracle.Chain(_workload(), n_threads=1)
    resumed.restore(blob)
    s0 = int(resumed.sweep[0])
    assert s0 % 7 == 0 and 21 <= s0 < total
    tail = resumed.run(total - s0)
    ref = oracle.Chain(_workload(), n_threads=1)
    head = ref.run(s0)
    rest = ref.run(total - s0)
    _same(_state(resumed), _state(ref))
    for k in ("e", "n", "state"):
        assert np.array_equal(tail[k], rest[k])
    assert len(head["n"]) > 0
