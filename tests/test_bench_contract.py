"""The benchmark's command-line contract (CPU): one GPU only, and the JSON fields the
roofline and baseline records carry.  The measurement itself runs on a GPU."""
import ast
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_result_record_names_the_contract_fields():
    src = open(os.path.join(ROOT, "bench.py")).read()
    tree = ast.parse(src)
    keys = {n.value for n in ast.walk(tree) if isinstance(n, ast.Constant) and isinstance(n.value, str)}
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "workload", "roofline", "bound", "achieved", "peak", "frac",
              "traffic", "cpu_baseline", "cores", "kind", "sample"):
        assert k in keys, k
