"""Host-side logic of bench.py (no GPU): the one-GPU guard, the CPU
baseline leg and the traffic table (the algorithmic byte counts behind
roofline.achieved are the library's own, checked on the GPU)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert "one GPU only" in out.stdout + out.stderr


def test_cpu_baseline_fields():
    """The oracle leg reports cell-updates/s on all host cores and on one,
    with the core count and the sample it timed (a tiny grid here)."""
    cb = bench.cpu_baseline(16)
    assert cb["kind"] == "oracle" and cb["unit"] == "cell-updates/s"
    assert cb["cores"] == bench.host_cores() >= 1
    assert cb["value"] > 0 and "16^3" in cb["sample"] and "status 0" in cb["sample"]
    if cb["cores"] > 1:
        assert cb["one_core"]["value"] > 0


def test_traffic_is_null_for_other_kernel_sources():
    """A PMC traffic figure is reported only for the kernel source it was
    measured on."""
    sha = bench.kernels_sha256()
    assert len(sha) == 64
    for key, tr in bench.PMC_TRAFFIC.items():
        assert len(key) == 3 and tr["bytes_per_launch"] > 0
