"""Host-side behaviour of bench.py that needs no GPU: the one-GPU guard and the
choice of the HBM-traffic figure per workload."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_figure_is_per_workload():
    b = _bench()
    assert b.measured_traffic("hubbard6") is None          # no counter summary for it
    for name in ("ueg57", "ueg123"):
        t = b.measured_traffic(name)
        # the summary's figure while the GEMM source is the one it was taken on, else none
        assert t is None or t > 0.0
    a, c = b.measured_traffic("ueg57"), b.measured_traffic("ueg123")
    if a is not None and c is not None:
        assert a != c
