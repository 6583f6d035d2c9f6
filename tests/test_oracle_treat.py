"""Pins of the oracle's gradient treatments (Sec. III-E) against what the
section fixes: clipping bounds every element and leaves the others alone,
scaling brings the rounded order of magnitude of the largest element down to
oom* by whole powers of ten, normalisation yields norm ||g|| / (||g|| + delta);
and brute force for the statistics of treated vectors."""
import math

import numpy as np
import pytest

from oracle import treatments as T


def _vectors(seed=3, n=40):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        size = int(rng.integers(1, 400))
        mag = 10.0 ** rng.uniform(-8, 14)
        g = rng.standard_normal(size) * mag
        if k % 5 == 0:
            g = np.abs(g)            # one-signed vectors
        if k % 7 == 0:
            g = -np.abs(g)
        out.append(g)
    return out


def test_clip_bounds_and_fixed_points():
    for g in _vectors():
        c = float(np.median(np.abs(g)))
        h = T.clip(g, c)
        assert np.all(np.abs(h) <= c)
        inside = np.abs(g) <= c
        assert np.array_equal(h[inside], g[inside])
        assert np.all(h[~inside] == np.sign(g[~inside]) * c)
    # the paper's threshold: a gradient of 3e7 becomes 1e4, one of -2.5 is kept
    assert list(T.clip(np.array([3e7, -2.5, -1e9]))) == [1e4, -2.5, -1e4]


def test_scale_worked_examples():
    # max |g| = 3.7e9: log10 = 9.57 rounds to 10, ten minus oom* 4 = 6 orders removed
    g = np.array([3.7e9, -1.0, 2.0])
    h = T.dynamic_scale(g, oom=4, delta=0.0)
    assert np.allclose(h, g / 1e6, rtol=1e-15)
    # max |g| = 1e8 exactly, delta 0: scaled to exactly 1e4
    assert T.dynamic_scale(np.array([-1e8, 5.0]), oom=4, delta=0.0)[0] == -1e4
    # a vector already at four orders of magnitude is left alone
    g = np.array([2.0e4, -3.0])
    assert np.array_equal(T.dynamic_scale(g, oom=4, delta=1e-6), g)
    # halves round away from zero: 10^4.5 rounds to order 5 and is scaled by 10
    g = np.array([10.0 ** 4.5 * (1 + 1e-12)])
    assert np.allclose(T.dynamic_scale(g, oom=4, delta=0.0), g / 10.0)
    assert T.round_half_away(-2.5) == -3.0 and T.round_half_away(2.5) == 3.0


def test_scale_bounds_order_of_magnitude():
    for g in _vectors(5):
        for oom in (0.0, 2.0, 4.0):
            h = T.dynamic_scale(g, oom=oom, delta=0.0)
            amax, hmax = np.max(np.abs(g)), np.max(np.abs(h))
            if T.round_half_away(math.log10(amax)) > oom:
                # whole powers of ten removed: the rounded order becomes oom*
                assert T.round_half_away(math.log10(hmax)) == oom
                ratio = g / h
                assert np.allclose(ratio, ratio[0], rtol=1e-12)
                k = math.log10(ratio[0])
                assert abs(k - round(k)) < 1e-9
            else:
                assert np.array_equal(h, g)


def test_normalise_norm_and_direction():
    for g in _vectors(7):
        n = np.linalg.norm(g)
        h = T.normalise(g, delta=1e-6)
        assert math.isclose(np.linalg.norm(h), n / (n + 1e-6), rel_tol=1e-12)
        cos = float(np.dot(g, h) / (np.linalg.norm(g) * np.linalg.norm(h)))
        assert math.isclose(cos, 1.0, rel_tol=1e-12)
    assert np.array_equal(T.normalise(np.zeros(4), delta=1e-6), np.zeros(4))


@pytest.mark.parametrize("mode", T.MODES)
def test_treated_stats_brute_force(mode):
    rng = np.random.default_rng(11)
    for g in _vectors(13):
        c = float(np.abs(g).max()) * rng.uniform(0.05, 1.5)
        got = T.treated_stats(*T.stats(g), mode, c=c, oom=3.0, delta=1e-6)
        want = T.stats(T.treat(g, mode, c=c, oom=3.0, delta=1e-6))
        assert math.isclose(got[0], want[0], rel_tol=1e-12, abs_tol=0.0)
        assert math.isclose(got[1], want[1], rel_tol=1e-12, abs_tol=0.0)
        if got[2] is not None:
            assert math.isclose(got[2], want[2], rel_tol=1e-12)
        else:
            assert mode == "clip" and want[2] <= T.stats(g)[2] * (1 + 1e-15)


def test_stats_of_empty_vector():
    assert T.stats(np.zeros(0)) == (0.0, 0.0, 0.0)
