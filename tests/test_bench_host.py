"""Host-side logic of bench.py (no GPU): the one-GPU guard and the
algorithmic byte model behind roofline.achieved."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert "one GPU only" in out.stdout + out.stderr


def test_smoother_class_bytes_v22_fp32():
    """V(2,2) in FP32 with the CG dots: first pair 6w, five half-sweeps 5w,
    the last half-sweep 4w + 24 B: 7 launches, 393 MB per launch at 256^3."""
    launches, b = bench.rbgs_fine_per_vcycle(2, 2, 4.0)
    assert launches == 7
    assert b == 6 * 4 + 5 * 5 * 4 + (4 * 4 + 24)
    assert round(b / launches * 256 ** 3) == 393066203


@pytest.mark.parametrize("pre,post", [(1, 1), (2, 2), (3, 1)])
def test_smoother_class_bytes_fp64(pre, post):
    launches, b = bench.rbgs_fine_per_vcycle(pre, post, 8.0)
    assert launches == 1 + 2 * (pre - 1) + 2 * post
    assert b == 6 * 8 + (launches - 1) * 5 * 8


def test_schur_bytes_by_precision():
    assert bench.class_bytes_per_cell("schur", 8.0) == 160.0
    assert bench.class_bytes_per_cell("schur", 4.0) == 176.0
    assert bench.class_bytes_per_cell("residual", 4.0) == 112.0
