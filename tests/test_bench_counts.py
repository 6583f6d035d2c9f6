"""The byte counts behind bench.py's two roofline figures, counted by hand
from what each step must read and write, and the one-GPU guard.  CPU only."""
import os
import subprocess
import sys

import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_p2g_bytes_by_hand():
    # 3D FP32: reads x, v, C, G (3 + 3 + 9 + 9 floats = 96 B), writes G' (36 B);
    # each active node (m > 0) receives m and mv (16 B)
    assert bench.algorithmic_bytes_p2g(1000, 170) == pytest.approx(1000 * (96 + 36) + 170 * 16)
    # 2D FP64: x, v, C, G = 2 + 2 + 4 + 4 doubles read (96 B), G' 4 doubles written; 3 doubles per node
    assert bench.algorithmic_bytes_p2g(100, 30, b=8, d=2) == pytest.approx(100 * (96 + 32) + 30 * 24)


def test_pass_bytes_by_hand():
    # per particle-step: state 96 B written and read in the forward (2x), in the
    # recompute (2x), read by the reverse step (1x), adjoint read and written
    # (2x); per active node in forward, recompute and reverse: m, mv written
    # and read (2 x 16 B) and v written and read (2 x 12 B)
    want = 7 * 96 + 3 * (2 * 16 + 2 * 12) * 1.3 / 8
    assert bench.algorithmic_bytes_pass(8000, 1300) == pytest.approx(want)
    assert want == pytest.approx(699.3)
    # 8 TB/s over those bytes
    assert bench.HBM_PEAK_GBS * 1e9 / want == pytest.approx(1.144e10, rel=1e-3)


def test_forward_bytes_by_hand():
    # per particle-step: state read and written (2 x 96 B); per active node m, mv
    # written and read (2 x 16 B) and v written and read (2 x 12 B)
    assert bench.algorithmic_bytes_forward(8000, 1300) == pytest.approx(2 * 96 + (2 * 16 + 2 * 12) * 1300 / 8000)
    assert bench.algorithmic_bytes_forward(8000, 1300) == pytest.approx(201.1)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
