"""Host-side checks of bench.py's contract pieces that need no GPU: it
refuses more than one GPU, and the measured HBM traffic it attaches to its
roofline entries comes from the committed counter summaries only for the
workload and kernel source they were taken on."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_source_digest_ignores_comments_and_layout(tmp_path):
    a = tmp_path / "a.hip"
    b = tmp_path / "b.hip"
    c = tmp_path / "c.hip"
    a.write_text("int f(int x) { return x + 1; }\n")
    b.write_text("// a comment\nint f(int x)\n{\n    /* another */ return x + 1;  // trailing\n}\n")
    c.write_text("int f(int x) { return x + 2; }\n")
    assert bench.kernel_source_digest(str(a)) == bench.kernel_source_digest(str(b))
    assert bench.kernel_source_digest(str(a)) != bench.kernel_source_digest(str(c))


def test_measured_traffic_only_for_the_profiled_workload():
    for kernel in ("k_sweep", "k_d2m"):
        assert bench.measured_traffic(kernel, "cfg2", "fp32") is None
        assert bench.measured_traffic(kernel, "cfg3", "fp64") is None
        t = bench.measured_traffic(kernel, "cfg3", "fp32")
        # a committed summary either matches the source (bytes per launch,
        # above the kernel's algorithmic bytes) or is reported as stale (None)
        assert t is None or t > 4.8e9
