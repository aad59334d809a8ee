"""Host-side checks of bench.py (no GPU): the one-GPU refusal, progress on
stderr only, and the algorithmic bytes per pixel and iteration that the
roofline divides by."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("model,n,ndim,storage,expect", [
    ("two", 2, 2, "f32", 48), ("two", 2, 2, "bf16", 28),
    ("potts", 4, 2, "f32", 152), ("potts", 4, 2, "bf16", 92),
    ("potts", 8, 2, "f32", 296), ("potts", 8, 2, "bf16", 180),
    ("two", 2, 3, "f32", 56), ("two", 2, 3, "bf16", 32)])
def test_algorithmic_bytes(model, n, ndim, storage, expect):
    """One read and one write of the state (u FP32; q, p_s, p / p_t in the
    storage type) and one read of the capacities: two-label (2d + 8)
    values, Potts (2d + 5) n + 2 values, at 4 or 2 bytes (u always 4)."""
    assert bench.alg_bytes(model, n, ndim, storage) == expect


def test_image_capacities_replace_the_planes():
    assert bench.alg_bytes("two", 2, 2, "f32", image=True) == 48 - 4
    assert bench.alg_bytes("potts", 8, 2, "f32", image=True) == 296 - 7 * 4


def test_progress_goes_to_stderr(capsys):
    """stdout carries only the JSON line; phase markers go to stderr."""
    bench.phase("headline: two_label_2d_2048 solves")
    out = capsys.readouterr()
    assert out.out == ""
    assert out.err == "[bench] headline: two_label_2d_2048 solves\n"
