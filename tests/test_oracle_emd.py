"""Pins of the oracle's earth mover's distance (Eq. emd): the assignment
against brute force over all injective maps and against scipy's linear-sum
assignment, the surface observation against a brute-force selection, closed
forms of the distance, and its gradient against central differences."""
import itertools
import math

import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

import workloads as W

RNG = np.random.default_rng(2024)


def _brute(cost):
    n, m = cost.shape
    best = math.inf
    for cols in itertools.permutations(range(m), n):
        best = min(best, sum(cost[i, c] for i, c in enumerate(cols)))
    return best


@pytest.mark.parametrize("n,m", [(1, 1), (2, 3), (4, 4), (5, 6), (3, 6)])
def test_assignment_brute_force(orc, n, m):
    for trial in range(20):
        cost = RNG.uniform(0, 1, (n, m))
        if trial % 4 == 0:
            cost = np.round(cost * 3)          # many ties
        col = orc.assign(cost)
        assert len(set(col.tolist())) == n and col.min() >= 0 and col.max() < m
        assert cost[np.arange(n), col].sum() == pytest.approx(_brute(cost), abs=1e-12)


@pytest.mark.parametrize("n,m", [(50, 50), (120, 200), (400, 400)])
def test_assignment_matches_scipy(orc, n, m):
    a = RNG.uniform(0, 1, (n, 3))
    b = RNG.uniform(0, 1, (m, 3))
    cost = np.linalg.norm(a[:, None, :] - b[None, :, :], axis=2)
    col = orc.assign(cost)
    r, c = linear_sum_assignment(cost)
    assert len(set(col.tolist())) == n
    assert cost[np.arange(n), col].sum() == pytest.approx(cost[r, c].sum(), rel=1e-13)


def test_surface_observation_brute_force(orc):
    w = W.tiny(3, shovel=True)
    cfg = orc.config(w)
    s = orc.initial_state(W.bed_positions(w))
    x = s[:, :3]
    x[:, 1] += RNG.uniform(0, 0.01, len(x))
    x[5, 1] = x[6, 1]                          # a tie in height
    got = orc.surface_particles(cfg, s)
    pix = w.hm_size / w.hm_res
    ix = np.floor((x[:, 0] - w.hm_origin[0]) / pix).astype(int)
    iz = np.floor((x[:, 2] - w.hm_origin[1]) / pix).astype(int)
    want = []
    for px in range(w.hm_res):
        for pz in range(w.hm_res):
            idx = np.nonzero((ix == px) & (iz == pz))[0]
            if len(idx):
                top = x[idx, 1].max()
                want.append(idx[x[idx, 1] == top].min())
    np.testing.assert_array_equal(got, want)


def _emd_config(orc, w, **over):
    return orc.config(w, w_hm=0.0, w_mass=0.0, **over)


def test_emd_closed_forms(orc):
    """Zero against the observed points themselves; a rigid shift t smaller
    than half the point spacing costs n |t| (the identity stays optimal)."""
    w = W.tiny(3, shovel=False, steps=1)
    w.w_emd = 1.0
    cfg = _emd_config(orc, w, gravity=0.0)
    s = orc.initial_state(W.bed_positions(w))
    surf = orc.surface_particles(cfg, s)
    pts = s[surf, :3].copy()
    # one sub-step with no gravity and no stress moves nothing
    p = w.params.copy()
    p[0] = 1e-9
    r = orc.rollout(cfg, p, s, 1, target=np.zeros(w.hm_res ** 2), emd_target=pts)
    assert r["loss"] == pytest.approx(0.0, abs=1e-12)
    t = np.array([0.002, -0.001, 0.0015])
    r = orc.rollout(cfg, p, s, 1, target=np.zeros(w.hm_res ** 2), emd_target=pts + t)
    assert r["loss"] == pytest.approx(len(pts) * np.linalg.norm(t), rel=1e-9)


def test_emd_loss_matches_scipy_on_the_final_state(orc):
    w = W.tiny(3, shovel=True, steps=40)
    w.w_emd = 0.7
    cfg = _emd_config(orc, w)
    s0 = orc.initial_state(W.bed_positions(w))
    tp = W.target_points(w, seed=5)
    r = orc.rollout(cfg, w.params, s0, 40, target=np.zeros(w.hm_res ** 2), emd_target=tp)
    surf = orc.surface_particles(cfg, r["state"])
    pts = r["state"][surf, :3]
    cost = np.linalg.norm(pts[:, None, :] - tp[None, :, :], axis=2)
    rr, cc = linear_sum_assignment(cost)
    assert r["loss"] == pytest.approx(0.7 * cost[rr, cc].sum(), rel=1e-12)


def test_emd_gradient_central_differences(orc):
    """d EMD / d params by forward mode against central differences (the
    assignment is locally constant, so the difference quotient is smooth)."""
    w = W.tiny(3, shovel=True, steps=20)
    w.w_emd = 1.0
    cfg = _emd_config(orc, w)
    s0 = orc.initial_state(W.bed_positions(w))
    tp = W.target_points(w, seed=7)
    zero = np.zeros(w.hm_res ** 2)
    r = orc.rollout(cfg, w.params, s0, 20, step0=150, target=zero, grad=True, emd_target=tp)
    g = r["grad"]
    for k in (0, 2, 4, 5, 6, 8):
        p = w.params
        errs = []
        for rel in (1e-5, 3e-6, 1e-6):
            h = rel * abs(p[k])
            lp = orc.rollout(cfg, np.where(np.arange(9) == k, p + h, p), s0, 20, step0=150, target=zero, emd_target=tp)["loss"]
            lm = orc.rollout(cfg, np.where(np.arange(9) == k, p - h, p), s0, 20, step0=150, target=zero, emd_target=tp)["loss"]
            fd = (lp - lm) / (2 * h)
            errs.append(abs(fd - g[k]) / (1e-6 * abs(fd) + 100 * np.finfo(float).eps * abs(r["loss"]) / h))
        assert min(errs) <= 1.0, (k, g[k], errs)
