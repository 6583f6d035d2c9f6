"""Test infrastructure (oracle): the gradient treatments of Sec. III-E applied
to whole gradient vectors in fp64, and the statistics of a vector that the
appendix on exploding gradients plots (largest and smallest element), plus the
2-norm.  Only the tests use this module; the library's reverse pass carries
its own implementation.

Readings of the section:
- "the largest element" of the scaling rule is read as the largest magnitude
  max |g|, the rule only ever reduces (it applies when the rounded order of
  magnitude exceeds oom*), and round() takes halves away from zero;
- a vector is one variable's adjoint for one simulation instance.

Parity pins (tests/test_oracle_treat.py): clipping bounds and fixed points,
the order of magnitude of scaled vectors, unit norm of normalised vectors, and
brute-force agreement of `treated_stats` with the statistics of treated
vectors.
"""
from __future__ import annotations

import math
from typing import Optional, Tuple

import numpy as np

MODES = ("none", "clip", "scale", "norm")

# Sec. III-E: the values used in the paper's experiments.
CLIP = 1e4
OOM = 4.0
DELTA = 1e-6


def round_half_away(x: float) -> float:
    return math.copysign(math.floor(abs(x) + 0.5), x)


def clip(g: np.ndarray, c: float = CLIP) -> np.ndarray:
    """Every element bounded to [-c, c]."""
    return np.minimum(np.maximum(g, -c), c)


def scale_exponent(amax: float, oom: float = OOM) -> float:
    """Delta oom of the scaling rule for a vector whose largest magnitude is
    amax: the rounded base-10 order of magnitude of amax minus oom*, 0 when
    the rule does not apply (amax zero or not finite, or already at most oom*
    orders of magnitude)."""
    if not (amax > 0.0) or math.isinf(amax):
        return 0.0
    d = round_half_away(math.log10(amax)) - oom
    return d if d > 0 else 0.0


def dynamic_scale(g: np.ndarray, oom: float = OOM, delta: float = DELTA) -> np.ndarray:
    """The vector divided by 10^d + delta, d = scale_exponent(max |g|)."""
    d = scale_exponent(float(np.max(np.abs(g))) if g.size else 0.0, oom)
    return g / (10.0 ** d + delta) if d > 0 else g.copy()


def normalise(g: np.ndarray, delta: float = DELTA) -> np.ndarray:
    """The vector divided by its 2-norm plus delta."""
    den = float(np.linalg.norm(g)) + delta
    return g / den if den > 0 else g.copy()


def treat(g: np.ndarray, mode: str, c: float = CLIP, oom: float = OOM, delta: float = DELTA) -> np.ndarray:
    g = np.asarray(g, dtype=np.float64)
    if mode == "none":
        return g.copy()
    if mode == "clip":
        return clip(g, c)
    if mode == "scale":
        return dynamic_scale(g, oom, delta)
    if mode == "norm":
        return normalise(g, delta)
    raise ValueError(mode)


def stats(g: np.ndarray) -> Tuple[float, float, float]:
    """(max, min, 2-norm) of a vector; zeros for an empty one."""
    g = np.asarray(g, dtype=np.float64).ravel()
    if g.size == 0:
        return 0.0, 0.0, 0.0
    return float(g.max()), float(g.min()), float(np.linalg.norm(g))


def treated_stats(mx: float, mn: float, nrm: float, mode: str, c: float = CLIP, oom: float = OOM,
                  delta: float = DELTA) -> Tuple[float, float, Optional[float]]:
    """Statistics of the treated vector from those of the vector: exact for
    max and min under every mode; the 2-norm is None under clipping, where it
    depends on more than the three numbers."""
    if mode == "none":
        return mx, mn, nrm
    if mode == "clip":
        return min(max(mx, -c), c), min(max(mn, -c), c), None
    if mode == "scale":
        d = scale_exponent(max(mx, -mn), oom)
        f = 1.0 / (10.0 ** d + delta) if d > 0 else 1.0
    elif mode == "norm":
        den = nrm + delta
        f = 1.0 / den if den > 0 else 1.0
    else:
        raise ValueError(mode)
    return mx * f, mn * f, nrm * f
