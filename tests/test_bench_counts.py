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
    # each occupied node (about 1.3 per cell of particles) receives m and mv (16 B)
    w = W.dig_3d(steps=10)
    n, ppc = w.n_particles, w.ppc
    assert bench.algorithmic_bytes_p2g([w]) == pytest.approx(n * (96 + 36) + 1.3 * n / ppc * 16)


def test_pass_bytes_by_hand():
    # per particle-step: state 96 B written and read in the forward (2x), in the
    # recompute (2x), read by the reverse step (1x), adjoint read and written
    # (2x); per occupied node in forward, recompute and reverse: m, mv written
    # and read (2 x 16 B) and v written and read (2 x 12 B)
    ws = W.sysid_batch(4, steps=10)
    assert all(w.ppc == 8 for w in ws)
    want = 7 * 96 + 3 * (2 * 16 + 2 * 12) * 1.3 / 8
    assert bench.algorithmic_bytes_pass(ws) == pytest.approx(want)
    assert want == pytest.approx(699.3)
    # 8 TB/s over those bytes
    assert bench.HBM_PEAK_GBS * 1e9 / want == pytest.approx(1.144e10, rel=1e-3)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
