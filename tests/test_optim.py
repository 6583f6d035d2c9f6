"""The optimiser driver (RMSprop with gradient clipping and a 5-candidate line
search, Sec. III-E, III-F, IV-B) on closed-form problems, without a GPU."""
import numpy as np
import pytest

from paper_2510_17335_amd import optim as O


def quad_problem(center, scale):
    center, scale = np.asarray(center, float), np.asarray(scale, float)

    def grad_fn(th):
        r = (th - center) / scale
        return float(np.sum(r * r)), 2.0 * r / scale

    def batch_fn(ths):
        return np.array([grad_fn(t)[0] for t in ths])
    return grad_fn, batch_fn


def test_first_rmsprop_step_is_step_over_sqrt_one_minus_beta():
    spec = O.OptimSpec(free=["E", "nu"], step={"E": 1e4, "nu": 0.01})
    g = np.array([3.0, -2e-3])
    v, d = O.rmsprop_direction(g, np.zeros(2), spec)
    np.testing.assert_allclose(v, 0.1 * g * g)
    # eps = 1e-8 in the denominator is 1.6e-5 of sqrt(v) for the second element
    np.testing.assert_allclose(d, np.array([1e4, -0.01]) / np.sqrt(0.1), rtol=1e-4)


def test_gradient_is_clipped_elementwise():
    spec = O.OptimSpec(free=["E"], step={"E": 1.0}, clip=1e4)
    v, _ = O.rmsprop_direction(np.array([5e7]), np.zeros(1), spec)
    np.testing.assert_allclose(v, 0.1 * 1e8)


def test_line_search_takes_the_best_candidate_and_respects_bounds():
    theta0 = np.array([1e5, 0.3, 30.0, 1600.0, 0.05, 30.0, 0.15])
    spec = O.OptimSpec(free=["E", "phi_deg"], step={"E": 1e4, "phi_deg": 1.0}, lo={"E": 9.5e4}, hi={"phi_deg": 31.0})
    seen = []

    def grad_fn(th):
        return 0.0, np.array([1.0, 0.0, -1.0, 0.0, 0.0, 0.0, 0.0])

    def batch_fn(ths):
        seen.extend(ths)
        return np.array([5.0, 1.0, 4.0, 3.0, 2.0])         # alpha 0.5 wins

    st = O.optimise(theta0, spec, grad_fn, batch_fn, 1)
    d = np.array([1e4, -1.0]) / np.sqrt(0.1)
    # candidates: theta - alpha d, clamped to E >= 9.5e4 and phi <= 31
    for a, th in zip(O.LINE_SEARCH, seen):
        assert th[0] == pytest.approx(max(1e5 - a * d[0], 9.5e4))
        assert th[2] == pytest.approx(min(30.0 - a * d[1], 31.0))
        np.testing.assert_array_equal(th[[1, 3, 4, 5, 6]], theta0[[1, 3, 4, 5, 6]])
    assert st.history[0]["chosen"] == 1
    np.testing.assert_array_equal(st.theta, seen[1])


def test_converges_on_a_separable_quadratic():
    center = np.array([2e5, 0.25, 35.0, 1800.0, 0.06, 20.0, 0.12, 0.03, 175.0])
    scale = np.array([1e5, 0.1, 10.0, 500.0, 0.03, 30.0, 0.1, 0.05, 20.0])
    grad_fn, batch_fn = quad_problem(center, scale)
    spec = O.OptimSpec(free=list(O.PARAM_NAMES),
                       step={"E": 1e4, "nu": 0.01, "phi_deg": 1.0, "rho": 50.0, **O.skill_steps()}, clip=1e30)
    theta0 = center + np.array([-8e4, 0.1, -8.0, -300.0, 0.02, 15.0, -0.05, -0.04, 12.0])
    st = O.optimise(theta0, spec, grad_fn, batch_fn, 60)
    losses = [h["loss"] for h in st.history]
    assert losses[-1] < 1e-2 * losses[0]
    # every accepted candidate is the best of its five
    for h in st.history:
        assert h["chosen"] == int(np.argmin(h["candidate_losses"]))


def test_skill_steps_follow_the_normalised_skill_mapping():
    s = O.skill_steps(0.03)
    # d2 = 0.03 (theta + 1), phi1 = theta pi/3 (in degrees 60 theta), d3 = 0.1 (theta + 1) + 0.04
    assert s["depth"] == pytest.approx(0.03 * 0.03)
    assert s["angle_deg"] == pytest.approx(np.degrees(np.pi / 3) * 0.03)
    assert s["push"] == pytest.approx(0.1 * 0.03)
    # d1 = 0.12 theta, phi3 = (theta + 3) pi/3 (in degrees 60 (theta + 3))
    assert s["displace"] == pytest.approx(0.12 * 0.03)
    assert s["push_angle_deg"] == pytest.approx(np.degrees(np.pi / 3) * 0.03)
