"""Pins of the oracle's per-step diagnostics (oracle.diagnostics) on the CPU:
closed forms for mass, momentum, kinetic energy and the CFL number of a
uniformly moving bed; the return-map case of every particle against a numpy
classification written from the yield condition of Eq. DP (singular values
from numpy's SVD, the material constants from their closed forms); the
clamp count; and the grid mass of a rollout against the particle mass
(each particle's B-spline weights sum to one)."""
import math

import numpy as np
import pytest

import workloads as W

RNG = np.random.default_rng(31)


def _material(E, nu, phi_deg):
    mu = E / (2 * (1 + nu))
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    s = math.sin(math.radians(phi_deg))
    return mu, lam, math.sqrt(2 / 3) * 2 * s / (3 - s)


def _cases(F, d, mu, lam, alpha):
    """Return-map case of each F (cohesionless): 1 tension (tr eps > 0), 2 inside
    the cone (|dev eps| + beta <= 0), 3 projection; beta = alpha (d lam + 2 mu)
    tr eps / (2 mu)."""
    out = []
    for f in F:
        eps = np.log(np.linalg.svd(f[:d, :d], compute_uv=False))
        tr = eps.sum()
        dev = eps - tr / d
        beta = alpha * (d * lam + 2 * mu) * tr / (2 * mu)
        out.append(1 if tr > 0 else (2 if np.linalg.norm(dev) + beta <= 0 else 3))
    return np.array(out)


def _state(x, v, F, d):
    n = x.shape[0]
    st = np.zeros((n, 2 * d + 2 * d * d))
    st[:, :d] = x
    st[:, d:2 * d] = v
    st[:, 2 * d + d * d:] = F[:, :d, :d].reshape(n, -1)
    return st


def _rotations(n):
    q, _ = np.linalg.qr(RNG.normal(size=(n, 3, 3)))
    return q * np.sign(np.linalg.det(q))[:, None, None]


@pytest.mark.parametrize("d", [2, 3])
def test_uniform_motion_closed_forms(orc, d):
    w = W.tiny(d, shovel=False)
    cfg = orc.config(w)
    x0 = W.bed_positions(w)
    n = x0.shape[0]
    v0 = np.array([0.3, -1.2, 0.5])[:d]
    F = np.tile(np.eye(3), (n, 1, 1))
    out = orc.diagnostics(cfg, w.params, _state(x0, np.tile(v0, (n, 1)), F, d))
    dx = 1.0 / w.n_grid
    m = n * w.params[3] * dx ** d / w.ppc
    assert out[0] == pytest.approx(m, rel=1e-14)
    np.testing.assert_allclose(out[1:1 + d], m * v0, rtol=1e-13)
    assert out[4] == pytest.approx(0.5 * m * float(v0 @ v0), rel=1e-13)
    assert out[9] == pytest.approx(np.abs(v0).max() * w.dt / dx, rel=1e-14)
    # F = I, C = 0: no strain, the elastic case for every particle
    assert list(out[5:9]) == [0, n, 0, 0]
    assert math.isnan(out[10])


@pytest.mark.parametrize("d", [2, 3])
def test_return_map_cases_against_numpy(orc, d):
    """Rotated diagonal strains of each kind, then a mixed set; C = 0, so
    F_tmp = F.  The numpy classification must give the intended case for the
    pure sets, and the oracle's counts must equal numpy's."""
    w = W.tiny(d, shovel=False)
    cfg = orc.config(w)
    E, nu, phi = w.params[:3]
    mu, lam, alpha = _material(E, nu, phi)
    x0 = W.bed_positions(w)
    n = x0.shape[0]
    R, Q = _rotations(n), _rotations(n)

    def F_of(eps):
        e = np.zeros((n, 3))
        e[:, :d] = eps
        S = np.zeros((n, 3, 3))
        S[:, np.arange(3), np.arange(3)] = np.exp(e)
        if d == 2:
            def rot2():
                a = RNG.uniform(0, 2 * np.pi, n)
                m = np.tile(np.eye(3), (n, 1, 1))
                m[:, 0, 0], m[:, 0, 1], m[:, 1, 0], m[:, 1, 1] = np.cos(a), -np.sin(a), np.sin(a), np.cos(a)
                return m
            return rot2() @ S @ rot2().transpose(0, 2, 1)
        return R @ S @ Q.transpose(0, 2, 1)

    sets = {
        1: RNG.uniform(0.001, 0.01, (n, d)),                                         # all stretched: tr > 0
        2: -0.01 + RNG.uniform(-1e-4, 1e-4, (n, d)),                                 # compressed, tiny deviator
        3: np.array([0.05, -0.08] if d == 2 else [0.05, -0.06, -0.02]) + RNG.uniform(-1e-3, 1e-3, (n, d)),
        # (3: compressed, |dev eps| about three times -beta)
    }
    v = np.zeros((n, d))
    for case, eps in sets.items():
        F = F_of(eps)
        ref = _cases(F, d, mu, lam, alpha)
        assert np.all(ref == case), (case, np.bincount(ref))
        out = orc.diagnostics(cfg, w.params, _state(x0, v, F, d))
        assert list(out[5:8]) == [n if k == case else 0 for k in (1, 2, 3)], (case, out[5:8])
        assert out[8] == 0
    mixed = np.concatenate([sets[1][: n // 3], sets[2][n // 3: 2 * n // 3], sets[3][2 * n // 3:]])
    RNG.shuffle(mixed)
    F = F_of(mixed)
    ref = _cases(F, d, mu, lam, alpha)
    out = orc.diagnostics(cfg, w.params, _state(x0, v, F, d))
    assert list(out[5:8]) == [int(np.sum(ref == k)) for k in (1, 2, 3)]


def test_clamped_singular_values_are_counted(orc):
    w = W.tiny(3, shovel=False)
    cfg = orc.config(w)
    x0 = W.bed_positions(w)
    n = x0.shape[0]
    F = np.tile(np.eye(3), (n, 1, 1))
    F[: n // 2, 2, 2] = 1e-8          # below the 1e-6 floor of the singular values
    out = orc.diagnostics(cfg, w.params, _state(x0, np.zeros((n, 3)), F, 3))
    assert out[8] == n // 2


@pytest.mark.parametrize("d", [2, 3])
def test_grid_mass_is_particle_mass(orc, d):
    w = W.tiny(d, shovel=(d == 3), steps=12)
    cfg = orc.config(w)
    r = orc.rollout(cfg, w.params, orc.initial_state(W.bed_positions(w)), 12, want_grid=True)
    out = orc.diagnostics(cfg, w.params, r["state"])
    assert r["grid"][:, 0].sum() == pytest.approx(out[0], rel=1e-13)


@pytest.mark.parametrize("d", [2, 3])
def test_cases_follow_the_trial_gradient(orc, d):
    """F = I and a velocity gradient C: the case is that of F_tmp = (I + dt C) F,
    not of F (which alone would be elastic); random velocities: the sums equal
    numpy's."""
    w = W.tiny(d, shovel=False)
    cfg = orc.config(w)
    E, nu, phi = w.params[:3]
    mu, lam, alpha = _material(E, nu, phi)
    x0 = W.bed_positions(w)
    n = x0.shape[0]
    v = RNG.normal(0, 0.5, (n, d))
    st = _state(x0, v, np.tile(np.eye(3), (n, 1, 1)), d)
    rate = 0.02 / w.dt                               # dt C = 0.02 I: a 2 % expansion
    st[:, 2 * d:2 * d + d * d] = (rate * np.eye(d)).reshape(-1)
    out = orc.diagnostics(cfg, w.params, st)
    Ft = np.tile(np.eye(3), (n, 1, 1))
    Ft[:, :d, :d] += w.dt * rate * np.eye(d)
    ref = _cases(Ft, d, mu, lam, alpha)
    assert np.all(ref == 1)
    assert list(out[5:8]) == [n, 0, 0]
    dx = 1.0 / w.n_grid
    mp = w.params[3] * dx ** d / w.ppc
    np.testing.assert_allclose(out[1:1 + d], mp * v.sum(0), rtol=1e-12, atol=1e-15)
    assert out[4] == pytest.approx(0.5 * mp * float((v * v).sum()), rel=1e-12)
    assert out[9] == pytest.approx(np.abs(v).max() * w.dt / dx, rel=1e-14)
