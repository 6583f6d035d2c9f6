"""The earth mover's distance term (Eq. emd) on the GPU against the oracle's
exact assignment, through the C-ABI: loss and gradients in FP64 on the tiny
bed, the 64^3 dig in FP32, and batched instances against single runs."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ddm():
    import torch
    assert torch.cuda.is_available()
    import paper_2510_17335_amd as m
    return m


def _run(ddm, w, steps, tg, tp, record=True, K=16):
    cfg, inst = ddm.from_workload(w, max_steps=steps, checkpoint_every=K)
    sim = ddm.Simulator(cfg, [inst])
    sim.set_emd_target(tp)
    sim.init_state(W.bed_positions(w))
    if record:
        sim.rollout(steps)
    else:
        sim.step(steps)
    loss = float(sim.loss(tg[None])[0])
    grad = sim.backward()[0].cpu().numpy() if record else None
    return loss, grad, sim.check()


@pytest.mark.parametrize("w_hm", [0.0, 1.0])
def test_emd_loss_and_gradient_tiny_f64(ddm, orc, w_hm):
    """EMD alone and with the height-map term: both sides solve the assignment
    exactly (the Hungarian method, ties to the lowest target), so the loss
    agrees to round-off and the 9 gradients to 1e-6."""
    w = W.tiny(3, shovel=True, steps=60)
    w.w_emd = 0.5
    w.w_hm = w_hm
    tg, tp = W.target_heightmap(w), W.target_points(w, seed=5)
    _log(f"case emd tiny3d f64 w_hm {w_hm}")
    loss, grad, err = _run(ddm, w, 60, tg, tp)
    r = orc.rollout(orc.config(w), w.params, orc.initial_state(W.bed_positions(w)), 60, target=tg, grad=True,
                    emd_target=tp)
    _log("gpu", loss, grad, "\noracle", r["loss"], r["grad"])
    assert err.flags == 0 and r["stats"][5] == 0
    assert abs(loss - r["loss"]) <= 1e-11 * abs(r["loss"]), loss - r["loss"]
    rel = np.abs(grad - r["grad"]) / np.maximum(np.abs(r["grad"]), 1e-9 * np.abs(r["grad"]).max())
    assert np.all(rel < 1e-6), rel


def test_emd_dig3d_f32(ddm, orc):
    """64^3 dig at 1 ppc (about 1400 observed points against 1600 targets),
    FP32, 100 sub-steps: the loss within 1e-4 of the FP64 oracle."""
    w = W.dig_3d(steps=100, ppc=1)
    w.w_emd = 1.0
    w.w_hm = 0.0
    w.w_mass = 0.0
    tg, tp = W.target_heightmap(w), W.target_points(w, seed=9)
    _log("case emd dig3d f32 ppc1 100 steps")
    loss, _, err = _run(ddm, w, 100, tg, tp, record=False)
    r = orc.rollout(orc.config(w), w.params, orc.initial_state(W.bed_positions(w)), 100, target=tg, emd_target=tp)
    _log("gpu", loss, "oracle", r["loss"])
    assert err.flags == 0 and err.clamp_count == 0 and r["stats"][0] == 0, (err.flags, r["stats"])
    assert abs(loss - r["loss"]) <= 1e-4 * abs(r["loss"])


def test_emd_batched_equals_single(ddm):
    """Two instances with their own targets in one context give the losses and
    gradients of two single-instance contexts (FP64)."""
    import torch
    w = W.tiny(3, shovel=True, steps=40)
    w.w_emd = 1.0
    tg = W.target_heightmap(w)
    tps = [W.target_points(w, seed=5), W.target_points(w, seed=6)]
    cfg, inst = ddm.from_workload(w, max_steps=40, checkpoint_every=16)
    from paper_2510_17335_amd import optim as O
    th2 = w.params.copy()
    th2[0] *= 1.5
    insts = [inst, O.instance_with(ddm, inst, th2)]
    sim = ddm.Simulator(cfg, insts)
    sim.set_emd_target(np.stack(tps))
    x0 = W.bed_positions(w)
    sim.init_state(np.concatenate([x0, x0]))
    sim.rollout(40)
    lb = sim.loss(np.stack([tg, tg])).cpu().numpy()
    gb = sim.backward().cpu().numpy()
    for i in range(2):
        s1 = ddm.Simulator(cfg, [insts[i]])
        s1.set_emd_target(tps[i])
        s1.init_state(x0)
        s1.rollout(40)
        l1 = float(s1.loss(tg[None])[0])
        g1 = s1.backward()[0].cpu().numpy()
        torch.cuda.synchronize()
        _log(f"instance {i}: batched {lb[i]} single {l1}")
        assert abs(lb[i] - l1) <= 1e-12 * abs(l1)
        np.testing.assert_allclose(gb[i], g1, rtol=1e-9, atol=1e-300)
