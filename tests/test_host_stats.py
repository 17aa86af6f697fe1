"""Host-side pieces of the benchmark (CPU only): the per-state efficiency ratio of
two time-to-accuracy runs, the single-GPU guard and the traffic figure's source
hash."""
from paper_1908_11118_amd.proposal import efficiency_ratio


def test_efficiency_ratio():
    a = {"se_by_state": [0.2, 0.4, 0.0], "t_acc_s": 10.0}
    b = {"se_by_state": [0.1, 0.4, 0.3], "t_acc_s": 20.0}
    r = efficiency_ratio(a, b)
    # 1/(SE^2 t): state 0 ratio (0.04*10)/(0.01*20) = 2, state 1 (0.16*10)/(0.16*20) = 0.5; state 2 frozen
    assert r["states"] == 2
    assert abs(r["max"] - 2.0) < 1e-12 and abs(r["min"] - 0.5) < 1e-12 and abs(r["geomean"] - 1.0) < 1e-12


def test_bench_refuses_more_than_one_gpu():
    """bench.py --gpus N > 1 prints one JSON line saying the run is single-GPU and exits 2."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


def test_bench_reports_traffic_only_for_the_profiled_sources(tmp_path, monkeypatch):
    """The committed counter summary applies while the kernel's sources (and the
    launch-shape code) hash to the profiled ones; any other hash gives no traffic."""
    import hashlib
    import os
    import bench
    h = hashlib.sha256()
    for f in bench.KERNEL_SOURCES:
        h.update(open(os.path.join(bench.ROOT, "paper_1908_11118_amd", "csrc", f), "rb").read())
    current = tmp_path / "current.md"
    current.write_text(f"# summary\n\nbytes_per_launch: 12345\nsource_sha256: {h.hexdigest()}\n")
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(current))
    assert bench.measured_traffic() == 12345.0
    stale = tmp_path / "stale.md"
    stale.write_text(f"bytes_per_launch: 12345\nsource_sha256: {'0' * 64}\n")
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(stale))
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(tmp_path / "missing.md"))
    assert bench.measured_traffic() is None
