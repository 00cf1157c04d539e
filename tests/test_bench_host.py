"""Host checks of bench.py's command-line contract (no GPU needed): more than one
GPU is refused with a message and exit status 2, and the algorithmic floor and
kernel grouping the roofline uses follow from the grid and nt alone."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


def test_floor_bytes_follow_the_compulsory_traffic_model():
    """32 V nt per Hessian-vector product (V = one vector field): 8.05 GB at 128^3,
    nt = 10, FP32; 4 V per stage launch; 4 V / 3 per transform pass."""
    import bench

    n = (128, 128, 128)
    V = 3 * 128 ** 3 * 4
    assert bench.hv_floor_bytes(n, 10, 4) == 32 * V * 10
    assert bench.floor_bytes_per_launch("tangent_stage", n, 4) == 4 * V
    assert bench.floor_bytes_per_launch("adjoint_stage", n, 4) == 4 * V
    assert abs(bench.floor_bytes_per_launch("fft_pencil_symbol", n, 4) - 4 * V / 3) <= 1


def test_kernel_groups_merge_predictor_and_corrector():
    import bench

    assert bench.kernel_group("tangent_stage_pred") == bench.kernel_group("tangent_stage_corr") == "tangent_stage"
    assert bench.kernel_group("tangent_stage_pred_first") == "tangent_stage"
    assert bench.kernel_group("adjoint_stage_corr_first") == "adjoint_stage"
    assert bench.kernel_group("fft_plane_inv_add") == bench.kernel_group("fft_plane_inv") == "fft_plane_inv"
