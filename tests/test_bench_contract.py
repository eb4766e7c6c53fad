"""The benchmark's contract pieces that need no GPU.

* `--gpus N` with N > 1 exits with status 2 and a message, before touching the
  GPU: the path runs on one GPU.
* The roofline's algorithmic flops per kernel evaluation, counted by hand: in
  2D the squared distance is 2 subtractions, 1 multiply and 1 multiply-add (5
  flops) and the contraction adds into 6 accumulator rows (lambda_i, i < 3,
  and the 3 products lambda_i lambda_j, i < j), one multiply-add each (12): 17.
  In 3D: 3 + 1 + 2 * 2 = 8 for the distance and 4 + 6 rows (20): 28.
"""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_flops_per_evaluation():
    sys.path.insert(0, ROOT)
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_contract", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    assert bench.flops_per_eval(2) == 17
    assert bench.flops_per_eval(3) == 28
    assert bench.FP32_VECTOR_PEAK_TFLOPS == 157.3
