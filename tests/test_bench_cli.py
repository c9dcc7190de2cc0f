"""bench.py on the host: it refuses more than one GPU before touching any,
and the counter figures it reports beside the live roofline (HBM bytes and
executed FP64 operations per evaluation) belong to the current EVALUATE
source and to a committed profile."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test",
                                                  os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_counter_figures_match_the_kernel_source():
    b = _bench()
    key = b.EVAL_TRAFFIC["kernel_sha256"]
    assert b._kernel_sha() == key, (
        "EVALUATE's source changed since its counters were taken: retake "
        "them (profiles/evaluate_gaussian_d5_counters.txt) and update the key")
    prof = os.path.join(ROOT, b.EVAL_TRAFFIC["profile"])
    text = open(prof).read()
    assert key in text
    # the executed FP64 operations per evaluation and the bytes per launch
    # are the profile's own figures
    assert "36.4 per evaluation" in text
    assert abs(b.EVAL_TRAFFIC["fp64_flop_per_eval"] - 36.4) < 0.05
    assert "39.38 MB per launch" in text
    assert abs(b.EVAL_TRAFFIC["bytes_per_launch"] / 1e6 - 39.38) < 0.005


def test_flop_table_covers_the_measured_workloads():
    b = _bench()
    text = open(os.path.join(ROOT, "profiles", "integrand_flops.txt")).read()
    for (family, d), flop in b.F_FLOP.items():
        row = [l for l in text.splitlines()
               if l.startswith(f"{family}_d{d} (d={d})")]
        assert len(row) == 1, (family, d)
        assert float(row[0].split()[6]) == flop, (family, d, row[0])
