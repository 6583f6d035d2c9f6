"""Pins of the oracle's full sub-step (Algorithm 1) and its gradient.

Invariants of MLS-MPM that hold exactly up to rounding (mass, linear and
angular momentum with the APIC affine term, the ballistic closed form, affine
field reproduction) and brute-force central differences of the loss on tiny
inputs.  CPU only.
"""
import math

import numpy as np
import pytest

import workloads as W



def _free_flight(orc, w, **over):
    """Configuration with no gravity, no container walls and no shovel."""
    return orc.config(w, shovel=False, gravity=0.0, bound=0, **over)


def _mass(w, rho):
    return rho * w.dx ** w.dim / w.ppc


@pytest.mark.parametrize("dim", [2, 3])
def test_mass_conservation(orc, dim):
    w = W.tiny(dim, shovel=(dim == 3))
    cfg = orc.config(w)
    s = orc.initial_state(W.bed_positions(w))
    mp = _mass(w, w.material.rho)
    for steps in (1, 7, 20):
        r = orc.rollout(cfg, w.params, s, steps, want_grid=True)
        assert r["grid"][:, 0].sum() == pytest.approx(mp * len(s), rel=1e-14)
        assert np.all(r["grid"][:, 0] >= 0)


def _random_motion(w, s, scale=0.2, seed=99):
    """A random affine motion plus per-particle noise, from its own seeded
    generator so that a test's input does not depend on which tests ran
    before it in the same process."""
    rng = np.random.default_rng(seed)
    d = w.dim
    n = s.shape[0]
    x = s[:, :d]
    v0 = rng.standard_normal(d) * scale
    A = rng.standard_normal((d, d)) * scale
    s = s.copy()
    s[:, d:2 * d] = v0 + x @ A.T + 0.05 * rng.standard_normal((n, d))
    s[:, 2 * d:2 * d + d * d] = (A + 0.5 * rng.standard_normal((n, d, d))).reshape(n, -1)
    return s


@pytest.mark.parametrize("dim", [2, 3])
def test_linear_and_angular_momentum_free_flight(orc, dim):
    """With g = 0 and no boundaries, sum m v and sum m (x x v + dx^2/4 axial(C))
    are conserved by P2G, the grid update and G2P + advection, stress included."""
    w = W.tiny(dim)
    cfg = _free_flight(orc, w)
    s = _random_motion(w, orc.initial_state(W.bed_positions(w)))
    d = w.dim
    mp = _mass(w, w.material.rho)

    def moments(st):
        x, v, Cm, F = orc.unpack(st, d)
        P = mp * v.sum(axis=0)
        k = w.dx ** 2 / 4
        if d == 2:
            L = mp * np.sum(x[:, 0] * v[:, 1] - x[:, 1] * v[:, 0] + k * (Cm[:, 1, 0] - Cm[:, 0, 1]))
        else:
            L = mp * (np.cross(x, v).sum(axis=0) + k * np.stack([
                Cm[:, 2, 1] - Cm[:, 1, 2], Cm[:, 0, 2] - Cm[:, 2, 0], Cm[:, 1, 0] - Cm[:, 0, 1]], 1).sum(axis=0))
        return P, L

    P0, L0 = moments(s)
    r = orc.rollout(cfg, w.params, s, 10)
    P1, L1 = moments(r["state"])
    assert np.max(np.abs(r["state"][:, 2 * d + d * d:] - s[:, 2 * d + d * d:])) > 1e-4  # F did change
    scale_p = mp * np.abs(s[:, d:2 * d]).sum()
    np.testing.assert_allclose(P1, P0, atol=1e-13 * scale_p)
    np.testing.assert_allclose(L1, L0, atol=1e-13 * scale_p)


@pytest.mark.parametrize("dim", [2, 3])
def test_ballistic_closed_form(orc, dim):
    """Uniform velocity under gravity, no walls: F stays I, C stays 0, and
    x_n = x_0 + n dt v_0 + dt^2 g n (n + 1) / 2 (symplectic Euler)."""
    w = W.tiny(dim)
    cfg = orc.config(w, shovel=False, bound=0)
    s = orc.initial_state(W.bed_positions(w))
    d = w.dim
    v0 = np.array([0.3, 0.5, -0.2][:d])
    s[:, d:2 * d] = v0
    n = 15
    r = orc.rollout(cfg, w.params, s, n)
    g = np.zeros(d)
    g[1] = w.gravity
    x_exp = s[:, :d] + n * w.dt * v0 + w.dt ** 2 * g * n * (n + 1) / 2
    np.testing.assert_allclose(r["state"][:, :d], x_exp, atol=1e-14)
    np.testing.assert_allclose(r["state"][:, d:2 * d], np.broadcast_to(v0 + n * w.dt * g, (len(s), d)), atol=1e-13)
    F = r["state"][:, 2 * d + d * d:].reshape(-1, d, d)
    np.testing.assert_allclose(F, np.broadcast_to(np.eye(d), F.shape), atol=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_affine_field_reproduction(orc, dim):
    """APIC with quadratic B-splines transfers an affine velocity field exactly:
    v_p = v0 + A x_p and C_p = A come back from one P2G + G2P (stress-free)."""
    w = W.tiny(dim)
    cfg = _free_flight(orc, w)
    s = orc.initial_state(W.bed_positions(w))
    d = w.dim
    rng = np.random.default_rng(5 + dim)
    v0 = rng.standard_normal(d) * 0.1
    A = rng.standard_normal((d, d)) * 0.1
    x = s[:, :d]
    s[:, d:2 * d] = v0 + x @ A.T
    s[:, 2 * d:2 * d + d * d] = A.reshape(-1)
    p = w.params.copy()
    p[0] = 1e-9                 # E ~ 0: no stress
    r = orc.rollout(cfg, p, s, 1)
    np.testing.assert_allclose(r["state"][:, d:2 * d], v0 + x @ A.T, atol=1e-13)
    Cm = r["state"][:, 2 * d:2 * d + d * d].reshape(-1, d, d)
    np.testing.assert_allclose(Cm, np.broadcast_to(A, Cm.shape), atol=1e-11)


def test_p2g_moments_single_particle(orc):
    """Quadratic B-spline identities through the P2G grid of one particle:
    sum w = 1, sum w (x_i - x_p) = 0, sum w (x_i - x_p)(x_i - x_p)^T = dx^2/4 I."""
    rng = np.random.default_rng(17)
    for dim in (2, 3):
        w = W.tiny(dim)
        cfg = orc.config(w, shovel=False, gravity=0.0, bound=0)
        for trial in range(5):
            x = rng.uniform(0.3, 0.7, size=(1, dim))
            s = orc.initial_state(x)
            r = orc.rollout(cfg, w.params, s, 1, want_grid=True)
            m = r["grid"][:, 0]
            mp = _mass(w, w.material.rho)
            idx = np.nonzero(m)[0]
            assert len(idx) == 3 ** dim
            coords = np.stack(np.unravel_index(idx, (w.n_grid,) * dim), 1) * w.dx
            wts = m[idx] / mp
            rr = coords - x[0]
            assert wts.sum() == pytest.approx(1.0, abs=1e-15)
            np.testing.assert_allclose(wts @ rr, 0.0, atol=1e-16)
            np.testing.assert_allclose((wts[:, None] * rr).T @ rr, np.eye(dim) * w.dx ** 2 / 4, atol=1e-17)


def _fd_grad(orc, cfg, params, s, steps, target, k, rel, step0=0):
    """Richardson-extrapolated central difference of the loss in parameter k
    (the step is relative to |p_k|, or to 0.05 m for a zero displacement)."""
    h = rel * (abs(params[k]) if params[k] != 0 else 0.05)

    def L(t):
        p = params.copy()
        p[k] += t
        return orc.rollout(cfg, p, s, steps, step0=step0, target=target)["loss"]

    d1 = (L(h) - L(-h)) / (2 * h)
    d2 = (L(2 * h) - L(-2 * h)) / (4 * h)
    return (4 * d1 - d2) / 3, h


@pytest.mark.parametrize("dim,shovel,step0,full", [(2, False, 0, False), (3, False, 0, False), (3, True, 0, False),
                                                   (3, True, 150, False), (3, True, 150, True)])
def test_gradient_matches_central_differences(orc, dim, shovel, step0, full):
    """Forward-mode gradient of the loss after 20 sub-steps vs brute-force
    central differences, for all 9 parameters (skill ones only with a shovel;
    step0 = 150 puts the insertion/push phases of the skill in the window;
    full: the unrounded skill mapping, particle-level collision, and a
    non-zero displacement and push angle away from pi).

    Contact and return-map branches make the loss piecewise smooth (a particle
    that changes return-map case a relative 2.5e-5 away from the point is
    common), so the difference quotient is taken at step sizes down to 1e-6
    relative and must agree at one of them to 1e-6 relative, beyond its own
    round-off floor 100 eps |L| / h."""
    w = W.tiny(dim, shovel=shovel)
    if w.target_seed is None:
        w.target_seed = 11
    if full:
        w.skill_unrounded = True
        w.particle_contact = True
        w.skill.displace = 0.02
        w.skill.push_angle_deg = 170.0
    cfg = orc.config(w)
    s = _random_motion(w, orc.initial_state(W.bed_positions(w)), scale=0.5)
    target = W.target_heightmap(w)
    r = orc.rollout(cfg, w.params, s, w.steps, step0=step0, target=target, grad=True)
    g, L = r["grad"], r["loss"]
    assert r["stats"][3] > 0               # plastic projections happened
    ks = range(9) if shovel else range(4)
    for k in ks:
        errs = []
        for rel in (1e-4, 3e-5, 1e-5, 3e-6, 1e-6):
            fd, h = _fd_grad(orc, cfg, w.params, s, w.steps, target, k, rel, step0)
            floor = 100 * np.finfo(float).eps * abs(L) / h
            errs.append(abs(g[k] - fd) / (1e-6 * abs(fd) + floor))
        assert min(errs) <= 1.0, (k, g[k], errs)
    if not shovel:
        assert np.all(g[4:] == 0)
    else:
        assert np.any(g[4:] != 0)
    if step0 == 150:
        assert g[4] != 0 and g[6] != 0        # depth (insertion) and push both act
    if full:
        assert g[7] != 0 and g[8] != 0        # displacement and push angle act


def _blade_at(orc, cfg, w, step):
    P, _ = orc.pose_table(cfg, w.params[4:9], w.dt, step + 1)
    return P[step]


def test_particle_collision_postcondition(orc):
    """Particle collision of Algorithm 1: after G2P every particle within the contact skin
    of the blade leaves it no faster than the blade along the normal
    ((v - v_s) . n >= 0), and particles in the wall layers are at rest.  The
    particle position of the test is the one before advection, x' - dt v'."""
    w = W.tiny(3, shovel=True, steps=170)
    w.particle_contact = True
    cfg = orc.config(w)
    s0 = orc.initial_state(W.bed_positions(w))
    hits = 0
    for n in (150, 165, 170):
        r = orc.rollout(cfg, w.params, s0, n)
        st = r["state"]
        x1, v1 = st[:, :3], st[:, 3:6]
        xp = x1 - w.dt * v1
        b = _blade_at(orc, cfg, w, n - 1)
        tip, psi, vel, om = b[:3], b[3], b[4:7], b[7]
        for q in range(xp.shape[0]):
            phi, nrm = orc.box_sdf(cfg, tip, psi, xp[q])
            if phi < w.skin:
                vs = np.array([vel[0] + om * (xp[q, 1] - tip[1]), vel[1] - om * (xp[q, 0] - tip[0]), vel[2]])
                assert np.dot(v1[q] - vs, nrm) >= -1e-12, (n, q)
                hits += 1
            if np.any(xp[q] < w.bound * w.dx) or np.any(xp[q] >= (w.n_grid - w.bound) * w.dx):
                assert np.all(v1[q] == 0.0)
    assert hits > 0


def test_particle_collision_changes_only_contacts(orc):
    """Without a blade near the bed and away from the walls the particle-level
    collision does nothing: the rollout is bit-identical with and without it;
    with the blade digging it changes the state."""
    w = W.tiny(3, shovel=False, steps=20)
    cfg_off = orc.config(w, bound=0)
    w.particle_contact = True
    cfg_on = orc.config(w, bound=0)
    s0 = _random_motion(w, orc.initial_state(W.bed_positions(w)), scale=0.1)
    a = orc.rollout(cfg_off, w.params, s0, 20)["state"]
    b = orc.rollout(cfg_on, w.params, s0, 20)["state"]
    np.testing.assert_array_equal(a, b)
    w2 = W.tiny(3, shovel=True, steps=170)
    c_off = orc.config(w2)
    w2.particle_contact = True
    c_on = orc.config(w2)
    s1 = orc.initial_state(W.bed_positions(w2))
    a = orc.rollout(c_off, w2.params, s1, 170)["state"]
    b = orc.rollout(c_on, w2.params, s1, 170)["state"]
    assert not np.array_equal(a, b)
