"""The optimiser driver on the GPU against a reference written here and
driven by the oracle, and the batched candidate evaluation against
one-instance runs."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ddm():
    import torch
    assert torch.cuda.is_available()
    import paper_2510_17335_amd as m
    return m


def _problem():
    w = W.tiny(3, shovel=True, steps=60)
    w.target_seed = 11
    return w, W.bed_positions(w), W.target_heightmap(w)


def test_optimiser_matches_an_oracle_driven_reference(ddm, orc):
    """Two RMSprop + line-search iterations on E, phi, depth and angle: the GPU
    evaluators inside the driver and the oracle inside a plain loop written
    here reach the same parameters and the same candidate losses."""
    from paper_2510_17335_amd import optim as O
    w, x0, tg = _problem()
    steps = 60
    free = ["E", "phi_deg", "depth", "angle_deg"]
    step = {"E": 2e4, "phi_deg": 2.0, **O.skill_steps()}
    theta0 = w.params.copy()
    ev = O.GpuEvaluator(ddm, w, x0, tg, steps, checkpoint_every=16, precision="f64")
    spec = O.OptimSpec(free=free, step=step, lo={"E": 1e4}, hi={"phi_deg": 60.0})
    st = O.optimise(theta0, spec, ev.grad, ev.losses, 2)

    # reference: the same update rules, evaluated by the oracle
    cfg = orc.config(w)
    s0 = orc.initial_state(x0)
    idx = [W_NAMES.index(n) for n in free]
    th, v = theta0.copy(), np.zeros(len(idx))
    for it in range(2):
        r = orc.rollout(cfg, th, s0, steps, target=tg, grad=True)
        g = np.clip(r["grad"][idx], -1e4, 1e4)
        v = 0.9 * v + 0.1 * g * g
        d = np.array([step[n] for n in free]) * g / (np.sqrt(v) + 1e-8)
        cands = []
        for a in (0.1, 0.5, 1.0, 1.5, 2.0):
            c = th.copy()
            c[idx] -= a * d
            c[0] = max(c[0], 1e4)
            c[2] = min(c[2], 60.0)
            cands.append(c)
        losses = np.array([orc.rollout(cfg, c, s0, steps, target=tg)["loss"] for c in cands])
        h = st.history[it]
        print(f"iteration {it}: gpu losses {h['candidate_losses']} oracle {losses}", flush=True)
        assert abs(h["loss"] - r["loss"]) <= 1e-9 * abs(r["loss"])
        np.testing.assert_allclose(h["candidate_losses"], losses, rtol=1e-8)
        best = int(np.argmin(losses))
        assert h["chosen"] == best
        th = cands[best]
        np.testing.assert_allclose(h["theta"], th, rtol=1e-7)


W_NAMES = ("E", "nu", "phi_deg", "rho", "depth", "angle_deg", "push")


def test_batched_candidates_equal_single_runs(ddm):
    """Losses of five parameter sets from one batched forward equal the losses
    of each run alone (FP64)."""
    from paper_2510_17335_amd import optim as O
    w, x0, tg = _problem()
    ev = O.GpuEvaluator(ddm, w, x0, tg, 60, checkpoint_every=16, precision="f64")
    rng = np.random.default_rng(3)
    thetas = []
    for k in range(7):                      # two launches, the second padded
        th = w.params.copy()
        th[0] *= 10 ** rng.uniform(-0.5, 0.5)
        th[2] += rng.uniform(-8, 8)
        th[4] *= rng.uniform(0.6, 1.4)
        thetas.append(th)
    batched = O.landscape(ev, thetas)
    single = np.array([ev.grad(th)[0] for th in thetas])
    print("batched", batched, "\nsingle ", single, flush=True)
    np.testing.assert_allclose(batched, single, rtol=1e-10)
