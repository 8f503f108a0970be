"""Host-side checks of bench.py: the one-GPU contract, the comment-blind code
hash that keys stored profiler measurements, and the lookup of measured HBM
traffic per launch."""

import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_code_hash_ignores_comments_and_whitespace(tmp_path):
    a = tmp_path / "a.h"
    b = tmp_path / "b.h"
    c = tmp_path / "c.h"
    a.write_text("int f(int x) { return x + 1; }\n")
    b.write_text("// increment\nint f(int x) {\n  /* one */ return x + 1;  // done\n}\n")
    c.write_text("int f(int x) { return x + 2; }\n")
    assert bench.code_hash(str(a)) == bench.code_hash(str(b))
    assert bench.code_hash(str(a)) != bench.code_hash(str(c))


def test_measured_traffic_lookup():
    assert bench.measured_traffic("no/such") is None
    for key in ("hvp/bwd", "c128:hvp/bwd"):
        v = bench.measured_traffic(key)
        # None when the sweep kernel changed since the counters were taken;
        # otherwise at least the 6 GiB the pass must move (4 slabs read, 2
        # written, 1 GiB each at the benchmark's chunk)
        assert v is None or v >= 0.9 * 6 * 2**30, (key, v)
    # Hessian sweeps (keyed on the Hessian kernel source): at least the
    # slices written per launch (8 slices x 2^15 rows x 1024 columns: 2 GiB
    # in complex64, 4 GiB in complex128; 6 slices with particle-number gates,
    # 1.5 GiB; configuration 4: 16 slices x 2^16 rows, 8 GiB)
    for key, least in (("cfg3:hess/sweep", 2 * 2**30), ("cfg3c128:hess/sweep", 4 * 2**30),
                       ("cfg3num:hess/sweep", 1.5 * 2**30), ("cfg4:hess/sweep", 8 * 2**30)):
        v = bench.measured_traffic(key, "hess")
        assert v is None or v >= 0.99 * least, (key, v)


def test_cpu_baseline_batches_over_workers():
    """The oracle baseline on a small problem: every sampled column is
    evaluated once, in batches over single-threaded worker processes, and
    the reported rate is the sample rate scaled to the full trace."""
    import workloads as w
    prob = w.make_problem(1)
    out = bench.cpu_baseline(prob, ncols=32, batch=8)
    assert out["kind"] == "oracle" and out["unit"] == "evals/s"
    assert out["value"] > 0 and 1 <= out["cores"] <= 16
    assert "32 basis states" in out["sample"] and "4 batches of 8" in out["sample"]
