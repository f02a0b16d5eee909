"""bench.py measures one GPU: asked for more it exits with a message before touching a
device (no GPU needed)."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_traffic_figures_follow_the_kernel_code(tmp_path):
    """The stored HBM traffic applies to the kernel code it was measured on: a comment edit
    keeps the code digest, a code edit changes it (and the traffic is then reported as
    null)."""
    sys.path.insert(0, ROOT)
    import bench
    src = tmp_path / "k.hip"
    src.write_text("// kernel\n__global__ void k(float* x) {  // one store\n    x[0] = 1.0f;\n}\n")
    d0 = bench.source_digest(str(src))
    src.write_text("// the kernel, reworded\n\n__global__ void k(float* x) {\n    x[0] = 1.0f;  // same\n}\n")
    assert bench.source_digest(str(src)) == d0
    src.write_text("__global__ void k(float* x) {\n    x[0] = 2.0f;\n}\n")
    assert bench.source_digest(str(src)) != d0
    # the figures of the profiled configurations (FFT tile length, P^T work range); none for
    # another configuration
    for name, cfg in (("ninv32", 16384), ("pt32", 512), ("ring_ninv32", 16384)):
        assert bench.kernel_traffic(name, cfg) is not None, name
    assert bench.kernel_traffic("ninv32", 8192) is None
