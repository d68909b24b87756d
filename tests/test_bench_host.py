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


def test_traffic_table_is_tied_to_the_measured_source():
    """A PMC traffic ratio is keyed by (class, mode, grid) and carries the
    hash of the kernel source it was measured on; the bench reports it only
    while the source hashes to that value."""
    sha = bench.kernels_sha256()
    assert len(sha) == 64
    for key, tr in bench.PMC_TRAFFIC.items():
        assert len(key) == 3 and key[0] in ("cg_vector", "spmv", "rbgs_fine")
        assert 0.5 < tr["ratio"] < 3.0 and len(tr["kernels_sha256"]) == 64
