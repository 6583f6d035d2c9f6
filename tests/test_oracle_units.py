"""Pins of the oracle's building blocks against the paper and the mathematics.

Each test checks the oracle against something other than itself: closed forms
printed in the paper, textbook identities, a library routine on a special case,
or brute force.  CPU only.
"""
import itertools
import math

import mpmath as mp
import numpy as np
import pytest

import workloads as W

RNG = np.random.default_rng(1234)


# --------------------------------------------------------------------------
# Skill-to-action mapping (Sec. III-B, Eqs. d1..delta_d4, Algorithm 2)
# --------------------------------------------------------------------------

def _closed_form_sums(th):
    """Sums over all actions and entries of d a / d theta with rounded T (the
    paper's Eqs. da-dtheta1-rounded .. da-dtheta5-rounded)."""
    phi1 = th[1] * math.pi / 3
    phi2 = phi1 + math.pi / 2
    d2 = (th[2] + 1) * 0.03
    d3 = (th[3] + 1) * 0.1 + 0.04
    phi3 = (th[4] + 3) * math.pi / 3
    return np.array([
        0.12,
        math.pi / 3 - d2 * math.pi / 3 * (math.sin(phi1 + math.pi / 2) + math.cos(phi1 + math.pi / 2)) - math.pi / 3,
        0.03 * (math.cos(phi2) - math.sin(phi2)),
        0.1 * (math.cos(phi3) + math.sin(phi3)),
        math.pi * d3 / 3 * (math.cos(phi3) - math.sin(phi3)),
    ])


@pytest.mark.parametrize("theta", [
    [0.3, 0.2, 0.8, -0.5, 0.0],          # demonstration skill (Sec. III-C) with a displacement
    [0.0, 0.5, 2.0 / 3.0, 0.1, 0.0],     # the 3D dig workload's skill
    [-0.4, -0.6, 0.15, 0.7, 0.4],
])
def test_skill_jacobian_sums_match_paper(orc, theta):
    T, acts, jac = orc.skill_actions(theta)
    sums = jac.sum(axis=(0, 1))
    np.testing.assert_allclose(sums, _closed_form_sums(theta), rtol=1e-12, atol=1e-14)
    # The same sums by central differences of the action values (T fixed).
    for k in range(5):
        h = 1e-6
        tp, tm = list(theta), list(theta)
        tp[k] += h
        tm[k] -= h
        Tp, ap, _ = orc.skill_actions(tp)
        Tm, am, _ = orc.skill_actions(tm)
        assert Tp == T and Tm == T
        fd = (ap.sum() - am.sum()) / (2 * h)
        assert abs(fd - _closed_form_sums(theta)[k]) < 1e-7


def test_skill_phase_lengths_by_hand(orc):
    # dt_action = 10 * 2e-4, v_l = 3 m/s, v_w = 10 pi rad/s:
    # phase 1: |pi/6| / (10 pi * 2e-3) = 8.33 -> 8; phase 2: 0.05 / 6e-3 = 8.33 -> 8;
    # phase 3: 0.15 / 6e-3 = 25 -> 25; phase 4: max(8.33, 0.01 / 6e-3) -> 8.
    T, acts, _ = orc.skill_actions([0.0, 0.5, 2.0 / 3.0, 0.1, 0.0])
    assert T == [8, 8, 25, 8]
    assert acts.shape == (49, 6)
    # Totals per phase equal the phase displacements (Eqs. delta_d1..delta_d4).
    assert abs(acts[:8, 3].sum() - math.pi / 6) < 1e-14
    assert abs(acts[8:16, 0].sum() - 0.05 * math.cos(math.pi / 6 + math.pi / 2)) < 1e-14
    assert abs(acts[8:16, 2].sum() + 0.05 * math.sin(math.pi / 6 + math.pi / 2)) < 1e-14
    assert abs(acts[16:41, 0].sum() + 0.15) < 1e-14
    assert abs(acts[41:, 3].sum() + math.pi / 6) < 1e-14
    assert abs(acts[41:, 2].sum() - 0.01) < 1e-14
    # FD of the dig skill at h = 1e-4 relative never crosses a rounding: every
    # T^float is at least 0.16 away from a half-integer.
    for tf in (8.333, 8.333, 25.0, 8.333):
        assert abs((tf % 1.0) - 0.5) > 0.16


def test_pose_table_follows_actions(orc):
    w = W.dig_3d()
    cfg = orc.config(w)
    P, J = orc.pose_table(cfg, [0.05, 30.0, 0.15, 0.0, 180.0], w.dt, 500)
    T, acts, _ = orc.skill_actions([0.0, 0.5, 2.0 / 3.0, 0.1, 0.0], dta=10 * w.dt)
    # After all 49 actions the tip moved by the summed displacement
    # (paper x, y, z -> build x, z, y) and psi returned to 0.
    tot = acts.sum(axis=0)
    expect = np.array(w.tip0) + np.array([tot[0], tot[2], tot[1]])
    np.testing.assert_allclose(P[489, :3], expect, atol=1e-14)
    assert abs(P[489, 3]) < 1e-14
    np.testing.assert_allclose(P[499, :3], P[489, :3], atol=0)
    assert np.all(P[490:, 4:] == 0)
    # After phase 2 the tip went d2 along the pointing direction e_p(phi1) = (-sin, -cos).
    d_ins = P[159, :3] - P[79, :3]
    np.testing.assert_allclose(d_ins, 0.05 * np.array([-math.sin(math.pi / 6), -math.cos(math.pi / 6), 0]), atol=1e-14)
    # velocity * dt equals the per-sub-step displacement
    np.testing.assert_allclose(P[1:490, :3] - P[:489, :3], P[1:490, 4:7] * w.dt, atol=1e-15)


def _phase_sums(jac, T):
    """Sums of d a / d theta over each phase's actions and all entries: [4, 5]."""
    b = np.cumsum([0] + list(T))
    return np.stack([jac[b[i]:b[i + 1]].sum(axis=(0, 1)) for i in range(4)])


def _fd_phase_sums(orc, theta, T, k, unrounded, h=1e-6, **kw):
    tp, tm = list(theta), list(theta)
    tp[k] += h
    tm[k] -= h
    Tp, ap, _ = orc.skill_actions(tp, unrounded=unrounded, **kw)
    Tm, am, _ = orc.skill_actions(tm, unrounded=unrounded, **kw)
    assert Tp == T and Tm == T
    b = np.cumsum([0] + list(T))
    return np.array([(ap[b[i]:b[i + 1]].sum() - am[b[i]:b[i + 1]].sum()) / (2 * h) for i in range(4)])


# Unrounded variant (Sec. III-B): phases 1 and 4 divide by T^float.  The
# paper's closed forms (Eqs. da-dtheta1-unrounded, da-dtheta2-unrounded and
# the two phase terms after it), with Delta t the action interval:
def _paper_unrounded(th, T, v_l, v_w, dta, d4):
    td, tr = th[0], th[1]
    Tf_d1, Tf_phi1 = abs(0.12 * td) / (v_l * dta), abs(tr * math.pi / 3) / (v_w * dta)
    Tf_lift = d4 / (v_l * dta)
    out = {}
    # d a[0:T1] / d theta_displace
    if Tf_d1 >= Tf_phi1 > 0 and td > 0:
        out["p1_displace"] = T[0] * (-math.pi * tr * v_l * dta / (0.36 * td ** 2))
    elif Tf_d1 >= Tf_phi1 > 0 and td < 0:
        out["p1_displace"] = T[0] * (2 * v_l * dta / td + math.pi * tr * v_l * dta / (0.36 * td ** 2))
    elif 0 < Tf_d1 < Tf_phi1:
        out["p1_displace"] = T[0] * 0.12 * v_w * dta / (abs(tr) * math.pi / 3)
    # d a[0:T1] / d theta_rotate
    if Tf_phi1 > Tf_d1 > 0 and tr > 0:
        out["p1_rotate"] = T[0] * (-0.36 * td * v_w * dta / (tr ** 2 * math.pi))
    elif Tf_phi1 > Tf_d1 > 0 and tr < 0:
        out["p1_rotate"] = T[0] * (2 * v_w * dta / tr + 0.36 * td * v_w * dta / (tr ** 2 * math.pi))
    elif 0 < Tf_phi1 <= Tf_d1:
        out["p1_rotate"] = T[0] * (math.pi / 3) * v_l * dta / (abs(td) * 0.12)
    # d a[T1+T2+T3:] / d theta_rotate
    if Tf_phi1 >= Tf_lift > 0 and tr > 0:
        out["p4_rotate"] = T[3] * (-3 * d4 * v_w * dta / (tr ** 2 * math.pi))
    elif Tf_phi1 >= Tf_lift > 0 and tr < 0:
        out["p4_rotate"] = T[3] * (-2 * v_w * dta / tr + 3 * d4 * v_w * dta / (tr ** 2 * math.pi))
    elif 0 < Tf_phi1 < Tf_lift:
        out["p4_rotate"] = T[3] * (-math.pi * v_l * dta / (3 * d4))
    # d a[T1:T1+T2] / d theta_rotate (T2 stays rounded)
    phi1 = tr * math.pi / 3
    out["p2_rotate"] = -(th[2] + 1) * 0.03 * math.pi / 3 * (math.sin(phi1 + math.pi / 2) + math.cos(phi1 + math.pi / 2))
    return out


@pytest.mark.parametrize("theta", [
    [0.6, 0.2, 0.3, -0.2, 0.1],      # phase 1 set by the displacement, theta > 0
    [0.1, 0.7, 0.8, 0.4, -0.3],      # phase 1 set by the rotation, theta > 0; phase 4 by the rotation
    [0.5, 0.05, 0.1, 0.0, 0.2],      # phase 4 set by the lift
    [-0.6, 0.2, 0.3, -0.2, 0.1],     # negative displacement
    [0.1, -0.7, 0.8, 0.4, -0.3],     # negative rotation
])
def test_unrounded_skill_jacobian(orc, theta):
    """Phase sums of the unrounded Jacobian against the paper's closed forms
    where theta_displace and theta_rotate are positive, and against central
    differences of the actions in every case.  For a negative theta the
    paper's expressions carry an extra 2 v dt / theta term; the derivative of
    the constant per-action step (-v dt) it would come from is zero, so the
    oracle follows the central differences there."""
    v_l, v_w, dta, d4 = 3.0, 10.0 * math.pi, 2e-3, 0.01
    T, acts, jac = orc.skill_actions(theta, v_l=v_l, v_w=v_w, dta=dta, d4=d4, unrounded=True)
    S = _phase_sums(jac, T)
    paper = _paper_unrounded(theta, T, v_l, v_w, dta, d4)
    got = {"p1_displace": S[0, 0], "p1_rotate": S[0, 1], "p4_rotate": S[3, 1], "p2_rotate": S[1, 1]}
    fd0 = _fd_phase_sums(orc, theta, T, 0, True)
    fd1 = _fd_phase_sums(orc, theta, T, 1, True)
    fds = {"p1_displace": fd0[0], "p1_rotate": fd1[0], "p4_rotate": fd1[3], "p2_rotate": fd1[1]}
    for key, g in got.items():
        assert abs(g - fds[key]) <= 1e-6 * max(1.0, abs(g)), (key, g, fds[key])
        neg = (key == "p1_displace" and theta[0] < 0) or (key in ("p1_rotate", "p4_rotate") and theta[1] < 0)
        if neg and key in paper:
            th = theta[0] if key == "p1_displace" else theta[1]
            v = v_l if key == "p1_displace" else v_w
            extra = 2 * v * dta / th * (T[0] if key != "p4_rotate" else -T[3])
            assert abs((paper[key] - extra) - g) <= 1e-9 * max(1.0, abs(g)), (key, paper[key], g, extra)
        elif key in paper:
            assert abs(paper[key] - g) <= 1e-9 * max(1.0, abs(g)), (key, paper[key], g)
    # phases 2 and 3 are those of the rounded mapping
    Tr, ar, jr = orc.skill_actions(theta, v_l=v_l, v_w=v_w, dta=dta, d4=d4)
    assert Tr == T
    b = np.cumsum([0] + list(T))
    np.testing.assert_array_equal(acts[b[1]:b[3]], ar[b[1]:b[3]])
    np.testing.assert_array_equal(jac[b[1]:b[3]], jr[b[1]:b[3]])


def test_unrounded_equals_rounded_at_integer_lengths(orc):
    """With T^float an integer the two mappings coincide: d1 / (v_l dta) = 4
    exactly for d1 = 0.024 m at v_l dta = 0.006 m; the rotation is shorter."""
    th = [0.2, 0.05, 0.3, 0.1, 0.0]
    T, a, _ = orc.skill_actions(th, unrounded=False)
    Tu, au, _ = orc.skill_actions(th, unrounded=True)
    assert T == Tu and T[0] == 4
    np.testing.assert_allclose(au[:4], a[:4], rtol=1e-15)


def test_pose_jacobian_of_new_skill_parameters(orc):
    """Columns of the pose Jacobian for the displacement and the push angle
    against central differences of the pose table."""
    w = W.dig_3d()
    cfg = orc.config(w)
    sk = np.array([0.05, 30.0, 0.15, 0.02, 170.0])
    P, J = orc.pose_table(cfg, sk, w.dt, 500)
    for k, h in ((3, 1e-6), (4, 1e-4)):
        sp, sm = sk.copy(), sk.copy()
        sp[k] += h
        sm[k] -= h
        Pp, _ = orc.pose_table(cfg, sp, w.dt, 500)
        Pm, _ = orc.pose_table(cfg, sm, w.dt, 500)
        np.testing.assert_allclose(J[:, :, k], (Pp - Pm) / (2 * h), atol=1e-7)
    assert np.any(J[:, :, 3] != 0) and np.any(J[:, :, 4] != 0)


# --------------------------------------------------------------------------
# SVD
# --------------------------------------------------------------------------

@pytest.mark.parametrize("d", [2, 3])
def test_svd_against_lapack(orc, d):
    for trial in range(200):
        F = np.eye(d) + 0.3 * RNG.standard_normal((d, d))
        if trial % 7 == 0:
            F = np.eye(d)
        if trial % 11 == 0:
            F = np.diag(RNG.uniform(0.5, 1.5, d))
            F[0, 0] = F[1, 1]          # repeated singular value
        U, S, V = orc.svd(F)
        np.testing.assert_allclose(U @ np.diag(S) @ V.T, F, atol=1e-13)
        np.testing.assert_allclose(U.T @ U, np.eye(d), atol=1e-13)
        np.testing.assert_allclose(V.T @ V, np.eye(d), atol=1e-13)
        assert np.linalg.det(U) > 0 and np.linalg.det(V) > 0
        ref = np.linalg.svd(F, compute_uv=False)
        got = np.sort(np.abs(S))[::-1]
        np.testing.assert_allclose(got, ref, rtol=1e-13)
        assert np.prod(S) * np.sign(np.linalg.det(F)) >= 0 or abs(np.linalg.det(F)) < 1e-12


def test_svd_inverted(orc):
    F = np.diag([1.2, 0.9, -0.8])
    U, S, V = orc.svd(F)
    np.testing.assert_allclose(U @ np.diag(S) @ V.T, F, atol=1e-14)
    assert (S < 0).sum() == 1 and np.argmin(S) == 2


# --------------------------------------------------------------------------
# SVK-Hencky elasticity (Eqs. SVK, piola): sigma = P F^T with det F' = 1
# --------------------------------------------------------------------------

def _psi(F, mu, lam):
    s = np.linalg.svd(F, compute_uv=False)
    e = np.log(s)
    return mu * np.sum(e * e) + 0.5 * lam * np.sum(e) ** 2


@pytest.mark.parametrize("d", [2, 3])
def test_stress_is_energy_derivative(orc, d):
    E, nu, phi = 3.5e5, 0.3, 30.0
    mu, lam, al, kc = orc.material(E, nu, phi)
    for trial in range(20):
        # compressive, nearly isotropic states stay inside the cone (elastic case)
        A = 0.01 * RNG.standard_normal((d, d))
        F = (1.0 - 0.02) * (np.eye(d) + A)
        cs, Fn, tau, _, _ = orc.constitutive(F, E, nu, phi)
        if cs != 2:
            continue
        # central differences of psi give P = d psi / d F (Eq. piola)
        P = np.zeros((d, d))
        h = 1e-7
        for i in range(d):
            for j in range(d):
                Fp, Fm = F.copy(), F.copy()
                Fp[i, j] += h
                Fm[i, j] -= h
                P[i, j] = (_psi(Fp, mu, lam) - _psi(Fm, mu, lam)) / (2 * h)
        np.testing.assert_allclose(Fn, F, atol=1e-14)
        np.testing.assert_allclose(tau, P @ F.T, rtol=1e-6, atol=1e-6 * np.abs(tau).max())


def test_lame_and_alpha(orc):
    mu, lam, al, kc = orc.material(3.5e5, 0.3, 30.0)
    assert mu == pytest.approx(3.5e5 / 2.6, rel=1e-15)
    assert lam == pytest.approx(3.5e5 * 0.3 / (1.3 * 0.4), rel=1e-15)
    s = math.sin(math.radians(30.0))
    assert al == pytest.approx(math.sqrt(2 / 3) * 2 * s / (3 - s), rel=1e-15)
    assert kc == 0.0


# --------------------------------------------------------------------------
# Drucker-Prager return map (Eq. DP) and App. B derivatives
# --------------------------------------------------------------------------

def _sample_sigma(d, n):
    return np.exp(RNG.normal(-0.01, 0.03, size=(n, d)))


@pytest.mark.parametrize("d", [2, 3])
def test_return_map_cases(orc, d):
    mu, lam, al, kc = orc.material(3.5e5, 0.3, 30.0)
    seen = set()
    for s in _sample_sigma(d, 3000):
        cs, g, h = orc.return_map(d, s, mu, lam, al)
        seen.add(cs)
        eps = np.log(s)
        ep = np.log(g)
        if cs == 1:
            assert eps.sum() > 0
            assert np.all(h == 0.0) and np.all(g == 1.0)
        elif cs == 2:
            np.testing.assert_allclose(g, s, rtol=1e-15)
        else:
            # lands on the cone: new delta_gamma = 0, trace kept, deviator shortened
            assert abs(orc.delta_gamma(d, g, mu, lam, al)) < 1e-12
            assert abs(ep.sum() - eps.sum()) < 1e-14
            dg = orc.delta_gamma(d, s, mu, lam, al)
            eh, eph = eps - eps.mean(), ep - ep.mean()
            assert abs(np.linalg.norm(eph) - (np.linalg.norm(eh) - dg)) < 1e-13
        # every output is inside the cone: ||dev tau|| + alpha tr tau <= 0, tr tau <= 0
        dev = h - h.mean()
        assert np.linalg.norm(dev) + al * h.sum() <= 1e-9 * (np.abs(h).max() + 1)
        assert h.sum() <= 1e-9
    assert seen == {1, 2, 3}


def test_return_map_appendix_b_derivatives(orc):
    """d delta_gamma / d mu and / d lambda (App. B) and dS'/d mu = dS'/d dgam * d dgam/d mu."""
    d = 3
    mu, lam, al, _ = orc.material(3.5e5, 0.3, 30.0)
    n_checked = 0
    for s in _sample_sigma(d, 400):
        cs, g, h = orc.return_map(d, s, mu, lam, al)
        if cs != 3:
            continue
        eps = np.log(s)
        tr = eps.sum()
        eh = eps - tr / d
        nrm = np.linalg.norm(eh)

        def dgam_from_output(m, l):
            c2, g2, _ = orc.return_map(d, s, m, l, al)
            assert c2 == 3
            ep = np.log(g2)
            return nrm - np.linalg.norm(ep - ep.mean())

        hm, hl = 1e-3 * mu, 1e-3 * lam
        fd_mu = (dgam_from_output(mu + hm, lam) - dgam_from_output(mu - hm, lam)) / (2 * hm)
        fd_lam = (dgam_from_output(mu, lam + hl) - dgam_from_output(mu, lam - hl)) / (2 * hl)
        assert fd_mu == pytest.approx(-lam * d * tr * al / (2 * mu ** 2), rel=1e-6)
        assert fd_lam == pytest.approx(d * tr * al / (2 * mu), rel=1e-6)
        dgam = nrm + (d * lam + 2 * mu) / (2 * mu) * tr * al
        dS_ddg = -np.exp(eps - dgam * eh / nrm) * eh / nrm
        g_p = orc.return_map(d, s, mu + hm, lam, al)[1]
        g_m = orc.return_map(d, s, mu - hm, lam, al)[1]
        np.testing.assert_allclose((g_p - g_m) / (2 * hm), dS_ddg * (-lam * d * tr * al / (2 * mu ** 2)),
                                   rtol=1e-5, atol=1e-16)
        n_checked += 1
    assert n_checked > 20


def test_cohesion_variant(orc):
    d = 3
    mu, lam, al, kc = orc.material(3.5e5, 0.3, 30.0, cohesion=500.0)
    assert kc > 0
    _, _, _, kc0 = orc.material(3.5e5, 0.3, 30.0, cohesion=0.0)
    assert kc0 == 0.0
    for s in _sample_sigma(d, 2000):
        cs, g, h = orc.return_map(d, s, mu, lam, al, kc)
        dev = h - h.mean()
        assert np.linalg.norm(dev) + al * h.sum() - kc <= 1e-9 * (np.abs(h).max() + kc)
        if cs == 1:
            # apex: isotropic, on the shifted apex tr tau = k_c / alpha
            assert abs(h.sum() - kc / al) < 1e-9 * kc / al
        # c = 0 gives the paper's map exactly
        c0, g0, h0 = orc.return_map(d, s, mu, lam, al, 0.0)
        c1, g1, h1 = orc.return_map(d, s, mu, lam, al)
        assert c0 == c1 and np.array_equal(g0, g1) and np.array_equal(h0, h1)


# --------------------------------------------------------------------------
# Tangents of the SVD-based constitutive update vs central differences
# --------------------------------------------------------------------------

def _near_apex(d, pair_gap):
    """F = Q diag(exp(eps)) Q^T on the cone just off its apex: a small negative
    trace, a deviator of ~1e-4 (3D) or ~6e-7 (2D), two strains pair_gap apart."""
    Q, _ = np.linalg.qr(RNG.standard_normal((d, d)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    if d == 3:
        eps = np.array([-1e-5 + 1e-4, -1e-5 + 1e-4 + pair_gap, -1e-5 - 2e-4 - pair_gap])
    else:
        eps = np.array([-1e-7 + pair_gap / 2, -1e-7 - pair_gap / 2])
    return Q @ np.diag(np.exp(eps)) @ Q.T


@pytest.mark.parametrize("d,gap", [(3, 3e-7), (3, 3e-9), (2, 8e-7)])
def test_constitutive_tangent_near_apex(orc, d, gap):
    """Near-isotropic plastic states (projection onto the cone, Eq. DP) with two
    close singular values: the SVD-frame derivative must use the divided
    difference of the return map, not its pointwise derivative."""
    E, nu, phi = 3.5e5, 0.3, 30.0
    for trial in range(5):
        F = _near_apex(d, gap)
        dF = RNG.standard_normal((d, d))
        cs, Fn, tau, dFn, dtau = orc.constitutive(F, E, nu, phi, dFt=dF)
        assert cs == 3
        h = 1e-7 if d == 3 else 2e-11

        def ev(t):
            c2, a, b, _, _ = orc.constitutive(F + t * dF, E, nu, phi)
            assert c2 == 3
            return a, b

        Fp, Tp = ev(h)
        Fm, Tm = ev(-h)
        Fp2, Tp2 = ev(2 * h)
        Fm2, Tm2 = ev(-2 * h)
        fdF = (8 * (Fp - Fm) - (Fp2 - Fm2)) / (12 * h)
        fdT = (8 * (Tp - Tm) - (Tp2 - Tm2)) / (12 * h)
        rt = 1e-5 if d == 3 else 1e-4
        np.testing.assert_allclose(dFn, fdF, rtol=rt, atol=rt * np.abs(fdF).max())
        np.testing.assert_allclose(dtau, fdT, rtol=rt, atol=rt * np.abs(fdT).max())


def _mp_update(F, d, mu, lam, alpha, kc):
    """F' = U diag(g) V^T and tau = U diag(h) U^T of one F_tmp in mpmath: the
    singular values from mpmath's own SVD, then the return map of Eq. DP on
    eps = ln s (with the cohesion shift) and the stress with det F' := 1."""
    U, S, Vt = mp.svd_r(F)
    s = [S[i] for i in range(d)]
    eps = [mp.log(x) for x in s]
    tr = mp.fsum(eps)
    dev = [e - tr / d for e in eps]
    nrm = mp.sqrt(mp.fsum([e * e for e in dev]))
    stiff = d * lam + 2 * mu
    tension = tr > 0 if kc == 0 else alpha * stiff * tr > kc
    if tension:
        ep, case = [kc / (d * alpha * stiff)] * d, 1
    else:
        dgam = nrm + stiff / (2 * mu) * tr * alpha - kc / (2 * mu)
        if dgam <= 0:
            ep, case = eps, 2
        else:
            ep, case = [e - dgam * x / nrm for e, x in zip(eps, dev)], 3
    tre = mp.fsum(ep)
    g = mp.diag([mp.exp(e) for e in ep])
    h = mp.diag([2 * mu * e + lam * tre for e in ep])
    return U * g * Vt, U * h * U.T, case


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("state", ["cone_apex", "cone", "elastic", "tension"])
@pytest.mark.parametrize("coh", [0.0, 500.0])
@pytest.mark.parametrize("gap", [1e-6, 3e-9, 1e-10, 1e-12, 1e-14, 0.0])
def test_constitutive_tangent_exact_near_ties(orc, d, state, coh, gap):
    """The SVD-frame tangent of F_tmp -> (F', tau) at close or tied singular
    values against the derivative of the same map evaluated at 80 digits
    (mpmath SVD, Eq. DP on ln s, central difference with step 1e-35).
    F_tmp is diagonal with decreasing entries, so the oracle's SVD frame is the
    identity exactly and the comparison sees only its divided differences.
    The strains are eps = (tr/d) 1 + dev with dev_0 - dev_1 = gap:
    "cone_apex": projection onto the cone (Eq. DP, third case) with a deviator
    as small as the gap, as for particles just off F = I (gap 3e-9 is a state
    where a two-point quadrature of the divided difference misses by several
    percent); "cone": the same case with a deviator of about 3e-3; "elastic":
    inside the cone; "tension": the apex case.  coh = 500 Pa shifts the cone
    (the cohesive variant), which puts the trace of the cone cases near the
    shifted apex."""
    E, nu, phi = 3.5e5, 0.3, 30.0
    mu, lam, alpha, kc = orc.material(E, nu, phi, coh)
    if d == 2 and gap == 0.0:
        pytest.skip("an exact tie in 2D leaves no deviator")
    g = gap if gap > 0 else 1e-9
    if state == "cone":
        raw = np.array([1e-3 + gap, 1e-3, -2e-3]) if d == 3 else np.array([gap, -2e-3])
    else:
        raw = np.array([g, 0.0 if gap > 0 else g, -1.5 * g]) if d == 3 else np.array([g, 0.0])
    dev = raw - raw.mean()
    nd = np.linalg.norm(dev)
    stiff = d * lam + 2 * mu
    tr = {"cone_apex": (kc - 0.3 * 2 * mu * nd) / (stiff * alpha),
          "cone": (kc - 0.3 * 2 * mu * nd) / (stiff * alpha),
          "elastic": (kc - 3.0 * 2 * mu * nd) / (stiff * alpha),
          "tension": kc / (stiff * alpha) + 1e-3}[state]
    s = np.exp(tr / d + dev)
    if gap == 0.0:
        s[1] = s[0]
    assert np.all(np.diff(s) <= 0)
    F = np.diag(s)
    rng = np.random.default_rng(abs(hash((d, state, coh, gap))) % 2**32)
    dF = rng.standard_normal((d, d))
    cs, Fn, tau, dFn, dtau = orc.constitutive(F, E, nu, phi, coh, dFt=dF)
    assert cs == {"cone_apex": 3, "cone": 3, "elastic": 2, "tension": 1}[state]
    def reference(Fd):
        with mp.workdps(80):
            mF = mp.matrix([[mp.mpf(float(v)) for v in row] for row in Fd])
            mdF = mp.matrix([[mp.mpf(float(v)) for v in row] for row in dF])
            mu_, lam_, al_, kc_ = (mp.mpf(float(v)) for v in (mu, lam, alpha, kc))
            h = mp.mpf("1e-35")
            Fp, Tp, cp = _mp_update(mF + h * mdF, d, mu_, lam_, al_, kc_)
            Fm, Tm, cm = _mp_update(mF - h * mdF, d, mu_, lam_, al_, kc_)
            _, _, c0 = _mp_update(mF, d, mu_, lam_, al_, kc_)
            assert cp == cm == c0 == cs, (cs, c0, cp, cm)
            rF = np.array([[float((Fp[i, j] - Fm[i, j]) / (2 * h)) for j in range(d)] for i in range(d)])
            rT = np.array([[float((Tp[i, j] - Tm[i, j]) / (2 * h)) for j in range(d)] for i in range(d)])
        return rF, rT

    rF, rT = reference(F)
    # Near the cohesive model's shifted apex (trace about 3e-3, deviator down
    # to 1e-14) the map itself is ill-conditioned in its FP64 inputs: the
    # trace's distance from the apex and the deviator are differences of
    # O(1e-3) logarithms.  There the bar is 1e-10 plus twice the change of the
    # exact derivative when each singular value moves by one ulp, which no
    # FP64 evaluation can go below.  Elsewhere the spread is far below 1e-10.
    sF, sT = np.zeros_like(rF), np.zeros_like(rT)
    if coh > 0 and state == "cone_apex":
        for signs in itertools.product((-1.0, 1.0), repeat=d):
            pF, pT = reference(np.diag(s * (1.0 + np.array(signs) * 2.0 ** -52)))
            sF, sT = np.maximum(sF, np.abs(pF - rF)), np.maximum(sT, np.abs(pT - rT))
    np.testing.assert_array_less(np.abs(dFn - rF), 1e-10 * np.abs(rF) + 2 * sF + 1e-12)
    np.testing.assert_array_less(np.abs(dtau - rT), 1e-10 * np.abs(rT) + 2 * sT + 1e-12 * max(1.0, np.abs(rT).max()))


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("kind", ["generic", "identity", "repeated", "plastic"])
def test_constitutive_tangent_vs_fd(orc, d, kind):
    E, nu, phi = 3.5e5, 0.3, 30.0
    n_ok = 0
    for trial in range(10):
        if kind == "generic":
            F = np.eye(d) + 0.05 * RNG.standard_normal((d, d))
        elif kind == "identity":
            F = np.eye(d)
        elif kind == "repeated":
            Q, _ = np.linalg.qr(RNG.standard_normal((d, d)))
            s = np.full(d, 0.97)
            if d == 3:
                s[2] = 0.99
            F = Q @ np.diag(s) @ Q.T
        else:
            F = np.eye(d) + 0.2 * RNG.standard_normal((d, d))
        dF = RNG.standard_normal((d, d))
        if kind == "identity":
            # F = I is the apex of the cone, where the three cases meet and the map
            # has no derivative; along rotations (skew dF) it is smooth: F' = I + t W.
            dF = dF - dF.T
        dp = RNG.standard_normal(3) * np.array([1e4, 0.01, 1.0])
        cs, Fn, tau, dFn, dtau = orc.constitutive(F, E, nu, phi, dFt=dF, dpar=dp)
        if cs < 0:
            continue

        def ev(t):
            c2, a, b, _, _ = orc.constitutive(F + t * dF, E + t * dp[0], nu + t * dp[1], phi + t * dp[2])
            return c2, a, b

        h = 1e-6
        c1, Fp, Tp = ev(h)
        c2, Fm, Tm = ev(-h)
        if kind != "identity" and not (c1 == cs == c2):
            continue     # a branch boundary lies within h
        c3, Fp2, Tp2 = ev(2 * h)
        c4, Fm2, Tm2 = ev(-2 * h)
        if kind != "identity" and not (c3 == cs == c4):
            continue
        # Richardson-extrapolated central differences
        fdF = (8 * (Fp - Fm) - (Fp2 - Fm2)) / (12 * h)
        fdT = (8 * (Tp - Tm) - (Tp2 - Tm2)) / (12 * h)
        np.testing.assert_allclose(dFn, fdF, rtol=1e-6, atol=1e-7 * (np.abs(fdF).max() + 1e-3))
        np.testing.assert_allclose(dtau, fdT, rtol=1e-6, atol=1e-7 * (np.abs(fdT).max() + 1.0))
        if kind == "identity":
            np.testing.assert_allclose(dFn, dF, atol=1e-12)
            np.testing.assert_allclose(dtau, 0.0, atol=1e-9)
        n_ok += 1
    assert n_ok >= 5


# --------------------------------------------------------------------------
# Shovel SDF and Coulomb contact
# --------------------------------------------------------------------------

def _box_brute(x, centre, axes, half, n=200):
    """Distance to the box boundary by dense sampling of its six faces."""
    best = np.inf
    g = np.linspace(-1, 1, n)
    A, B = np.meshgrid(g, g, indexing="ij")
    for f in range(3):
        a, b = [k for k in range(3) if k != f]
        for sgn in (-1, 1):
            pts = (centre[None, :] + sgn * half[f] * axes[f][None, :]
                   + (A.reshape(-1, 1) * half[a]) * axes[a][None, :]
                   + (B.reshape(-1, 1) * half[b]) * axes[b][None, :])
            best = min(best, np.min(np.linalg.norm(pts - x[None, :], axis=1)))
    return best


def test_box_sdf_brute_force(orc):
    w = W.dig_3d()
    cfg = orc.config(w)
    half = np.array(w.shovel_half)
    for trial in range(30):
        tip = np.array([0.5, 0.3, 0.5]) + 0.01 * RNG.standard_normal(3)
        psi = RNG.uniform(-0.6, 0.6)
        ep = np.array([-math.sin(psi), -math.cos(psi), 0.0])
        en = np.array([math.cos(psi), -math.sin(psi), 0.0])
        ew = np.array([0.0, 0.0, 1.0])
        centre = tip - half[2] * ep
        x = centre + RNG.uniform(-0.07, 0.07, 3)
        phi, nrm = orc.box_sdf(cfg, tip, psi, x)
        loc = np.array([np.dot(x - centre, e) for e in (ew, en, ep)])
        inside = np.all(np.abs(loc) <= half)
        dist = _box_brute(x, centre, [ew, en, ep], half)
        # sampling error: at most half the diagonal of one sample cell
        assert abs(abs(phi) - dist) < 3.5e-4
        assert (phi < 0) == inside
        if not inside:
            # exact: distance to the closest point of the solid box (clamped local coordinates)
            assert abs(phi - np.linalg.norm(loc - np.clip(loc, -half, half))) < 1e-15
        assert abs(np.linalg.norm(nrm) - 1) < 1e-12
        # the normal is the SDF gradient (central differences), off the medial axes
        h = 1e-7
        g = np.array([(orc.box_sdf(cfg, tip, psi, x + h * e)[0] - orc.box_sdf(cfg, tip, psi, x - h * e)[0]) / (2 * h)
                      for e in np.eye(3)])
        if not inside:
            np.testing.assert_allclose(g, nrm, atol=1e-6)


def test_coulomb_cases(orc):
    n = np.array([0.0, 1.0, 0.0])
    vs = np.array([0.1, 0.0, 0.0])
    # separating: unchanged
    v = orc.coulomb(vs, n, 0.5, [0.3, 0.2, 0.0])
    np.testing.assert_array_equal(v, [0.3, 0.2, 0.0])
    # sticking: |v_t| = 0.1 <= 0.5 * 1.0 -> rigid velocity
    v = orc.coulomb(vs, n, 0.5, [0.2, -1.0, 0.0])
    np.testing.assert_allclose(v, vs, atol=1e-15)
    # slipping: v_rel = (2, -1, 0): v_t = (2,0,0), reduced by mu |v_n| = 0.5
    v = orc.coulomb(vs, n, 0.5, [2.1, -1.0, 0.0])
    np.testing.assert_allclose(v, vs + np.array([1.5, 0.0, 0.0]), atol=1e-15)
    # frictionless: tangential part kept, normal part removed
    v = orc.coulomb(vs, n, 0.0, [0.7, -1.0, 0.4])
    np.testing.assert_allclose(v, [0.7, 0.0, 0.4], atol=1e-15)


# --------------------------------------------------------------------------
# Binning: keys and stable permutation (properties that pin them)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("d,tile", [(2, 4), (3, 4), (3, 8)])
def test_bin_keys_properties(orc, d, tile):
    n_grid = 64
    x = RNG.uniform(0.05, 0.95, size=(5000, d))
    x[::7] = x[::7][:, :]                      # keep some duplicates of cells
    x[1::50] = x[0::50][: len(x[1::50])]       # exact duplicates: ties
    inst = (np.arange(len(x)) % 3).astype(np.int32)
    keys, perm = orc.bin_keys(x, n_grid, tile, inst)
    assert sorted(perm.tolist()) == list(range(len(x)))
    ks = keys[perm]
    assert np.all(np.diff(ks.astype(np.int64)) >= 0)
    same = np.diff(ks.astype(np.int64)) == 0
    assert np.all(np.diff(perm.astype(np.int64))[same] > 0)      # stable
    cells = n_grid ** d
    nt = n_grid // tile
    for p in range(0, len(x), 97):
        k = int(keys[p])
        assert k // cells == inst[p]
        loc = k % cells
        t, c = divmod(loc, tile ** d)
        base = []
        for a in reversed(range(d)):
            base.append((t % nt) * tile + c % tile)
            t //= nt
            c //= tile
        base = np.array(base[::-1])
        f = x[p] * n_grid - base
        assert np.all(f >= 0.5) and np.all(f < 1.5)
