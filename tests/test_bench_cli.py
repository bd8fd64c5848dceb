"""Command-line contract of bench.py that needs no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_printed_line_is_strict_json():
    """Identical gated and plain images give an infinite PSNR; the line
    carries null there instead of the non-standard `Infinity`."""
    import importlib.util
    import json
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    assert bench.psnr_db(0.0) is None
    assert abs(bench.psnr_db(1e-4) - 40.0) < 1e-12
    line = json.dumps(bench.finite({"psnr": float("inf"), "rows": [{"x": float("nan")}, 1.5]}), allow_nan=False)
    assert json.loads(line) == {"psnr": None, "rows": [{"x": None}, 1.5]}


def test_host_cpu_reports_model_and_counts():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    model, n_cpu, n_avail = bench.host_cpu()
    assert isinstance(model, str) and model
    assert n_cpu >= 1 and 1 <= n_avail <= n_cpu
