"""Gradient treatments inside the reverse pass (Sec. III-E) and the record of
adjoint growth, through the C-ABI.

Treated gradients are not derivatives of the loss, so the forward-mode oracle
has no counterpart for them; the checks are:
- the record leaves the gradient as it was, and its statistics are
  consistent (max >= min, norm >= the largest magnitude);
- thresholds that never act (clip 1e30, oom* 300) leave the gradient as it
  was;
("as it was": within the spread of two untreated passes, whose FP64 atomic
sums may add in a different order: 1e-10 relative in FP64, 1e-4 in FP32);
- the record of a pass repeats in FP32, whose forward pass is bitwise
  repeatable.  In FP64 the order of the atomic sums moves the state by about
  1e-15, and a bed that starts at rest has every particle at F = I, on the
  boundary of the cone-tip case of the return map (tr(log sigma) = 0): such a
  particle takes either case from one run to the next, which changes its F
  adjoint by O(1) in the first sub-steps while its stress, and with it the
  parameter gradient, stays within round-off;
- thresholds that act: per sub-step, instance and variable, the statistics
  after the treatment equal the oracle's statistics of the treated vector
  computed from those before it, and the gradient moves;
- instances stay independent: each instance of a batch gets the treated
  gradient and statistics it gets alone;
- a captured pass (HIP graph) gives the gradient of the eager pass.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import treatments as OT

pytestmark = pytest.mark.gpu

STEPS = 60


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ddm():
    import torch
    assert torch.cuda.is_available()
    import paper_2510_17335_amd as m
    return m


def _sim(ddm, precision, thetas=None, steps=STEPS):
    from paper_2510_17335_amd import optim as O
    w = W.dig_3d(steps=steps)
    cfg, inst = ddm.from_workload(w, max_steps=steps, checkpoint_every=16, precision=precision)
    insts = [inst] if thetas is None else [O.instance_with(ddm, inst, th) for th in thetas]
    sim = ddm.Simulator(cfg, insts)
    x0 = W.bed_positions(w)
    tg = W.target_heightmap(w).reshape(1, -1)
    return w, sim, np.concatenate([x0] * len(insts)), np.repeat(tg, len(insts), axis=0)


def _grad(sim, x0, tg, steps=STEPS):
    sim.init_state(x0)
    sim.rollout(steps)
    sim.loss(tg)
    g = sim.backward().cpu().numpy()
    e = sim.check()
    assert e.flags & 1 == 0, "NaN or Inf on the device"
    return g


def _same(a, b, precision, what):
    rel = float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))
    _log(f"{what}: max relative difference {rel:.3e}")
    assert rel <= (1e-10 if precision == "f64" else 1e-4), (what, rel)


def _same_record(a, b, precision, what):
    """Records agree to the tolerance of _same relative to each vector's
    2-norm: an extreme of a one-signed vector can be a round-off-sized number
    whose relative spread says nothing."""
    scale = np.concatenate([np.repeat(b[..., 2:3], 3, axis=-1), np.repeat(b[..., 5:6], 3, axis=-1)], axis=-1)
    rel = np.abs(a - b) / np.maximum(scale, 1e-300)
    at = np.unravel_index(int(np.argmax(rel)), rel.shape)
    _log(f"{what}: max difference {float(rel[at]):.3e} of the vector norm at {at}: {a[at]!r} vs {b[at]!r}")
    assert float(rel[at]) <= (1e-10 if precision == "f64" else 1e-4), (what, at)


def _check_stats_consistent(S):
    pre = S[..., :3]
    assert np.all(np.isfinite(S))
    assert np.all(pre[..., 0] >= pre[..., 1])
    amax = np.maximum(np.abs(pre[..., 0]), np.abs(pre[..., 1]))
    assert np.all(pre[..., 2] >= amax * (1 - 1e-12))


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_record_keeps_gradient_and_is_consistent(ddm, precision):
    _log(f"case record f={precision} dig3d 64^3 {STEPS} steps")
    w, sim, x0, tg = _sim(ddm, precision)
    g0 = _grad(sim, x0, tg)
    sim.set_grad_treatment("none", record_steps=STEPS)
    g1 = _grad(sim, x0, tg)
    _same(g1, g0, precision, "gradient with the record")
    S = sim.grad_stats()
    assert S.shape == (STEPS, 1, 6, 6)
    _check_stats_consistent(S)
    assert np.array_equal(S[..., :3], S[..., 3:])
    # every variable has a non-zero adjoint over the horizon
    assert np.all(S[..., 2].max(axis=0) > 0)
    # the record is rewritten by every backward pass
    g2 = _grad(sim, x0, tg)
    _same(g2, g0, precision, "second pass")
    if precision == "f32":
        _same_record(sim.grad_stats(), S, precision, "second record")
    _log("norms of x-bar at steps 0, mid, last:", S[0, 0, 0, 2], S[STEPS // 2, 0, 0, 2], S[-1, 0, 0, 2])
    # growth per checkpoint segment: maxima over the segment's sub-steps
    G = sim.grad_growth()
    S = sim.grad_stats()
    assert G.shape == ((STEPS + 15) // 16, 1, 6, 2)
    amax = np.maximum(np.abs(S[..., 0]), np.abs(S[..., 1]))
    for q in range(G.shape[0]):
        assert np.array_equal(G[q, ..., 0], amax[16 * q:16 * (q + 1)].max(axis=0))
        assert np.array_equal(G[q, ..., 1], S[16 * q:16 * (q + 1), ..., 2].max(axis=0))


def test_idle_thresholds_keep_gradient(ddm):
    _log("case idle thresholds f32")
    w, sim, x0, tg = _sim(ddm, "f32")
    g0 = _grad(sim, x0, tg)
    sim.set_grad_treatment("clip", clip=1e30)
    _same(_grad(sim, x0, tg), g0, "f32", "clip 1e30")
    sim.set_grad_treatment("scale", oom=300.0)
    _same(_grad(sim, x0, tg), g0, "f32", "oom* 300")
    sim.set_grad_treatment("none")
    _same(_grad(sim, x0, tg), g0, "f32", "none")


def _acting_thresholds(S):
    """A clip threshold (a power of two, exact in FP32) and an oom* that act on
    about half of the recorded vectors."""
    amax = np.maximum(np.abs(S[..., 0]), np.abs(S[..., 1])).ravel()
    amax = amax[amax > 0]
    med = float(np.median(amax))
    return 2.0 ** np.floor(np.log2(med)), float(np.round(np.log10(med)))


@pytest.mark.parametrize("precision", ["f32", "f64"])
@pytest.mark.parametrize("mode", ["clip", "scale", "norm"])
def test_treatment_statistics_match_oracle(ddm, precision, mode):
    _log(f"case treat {mode} f={precision}")
    w, sim, x0, tg = _sim(ddm, precision)
    sim.set_grad_treatment("none", record_steps=STEPS)
    g0 = _grad(sim, x0, tg)
    c, oom = _acting_thresholds(sim.grad_stats())
    delta = 1e-6
    sim.set_grad_treatment(mode, clip=c, oom=oom, delta=delta, record_steps=STEPS)
    g1 = _grad(sim, x0, tg)
    S = sim.grad_stats()
    _check_stats_consistent(S)
    rtol = 2e-6 if precision == "f32" else 1e-13
    acted = 0
    for k in range(STEPS):
        for v in range(6):
            pre, post = S[k, 0, v, :3], S[k, 0, v, 3:]
            want = OT.treated_stats(*pre, mode, c=c, oom=oom, delta=delta)
            for a in range(3):
                if want[a] is None:
                    assert post[a] <= pre[a] * (1 + 1e-12)
                    continue
                assert abs(post[a] - want[a]) <= rtol * abs(want[a]) + 1e-300, (k, OT_VARS[v], a, post, want)
            acted += int(not np.array_equal(pre, post))
    _log(f"{mode}: {acted} of {STEPS * 6} vectors changed; grad {g1[0]} (untreated {g0[0]})")
    assert acted > 0
    assert np.all(np.isfinite(g1)) and not np.array_equal(g0, g1)


OT_VARS = ("x", "v", "F", "grid_v_post", "grid_mv", "grid_m")


def test_batched_instances_are_treated_alone(ddm):
    """Two instances with different parameters in one batch against each alone
    (normalisation, FP32): per-instance vectors, so identical up to the
    summation order of the reductions."""
    _log("case treat norm batched vs alone f32")
    w = W.dig_3d(steps=STEPS)
    th = [w.params.copy(), w.params.copy()]
    th[1][0] *= 1.7
    th[1][5] += 6.0
    _, bsim, x0b, tgb = _sim(ddm, "f32", th)
    bsim.set_grad_treatment("norm", record_steps=STEPS)
    gb = _grad(bsim, x0b, tgb)
    Sb = bsim.grad_stats()
    for i in range(2):
        _, sim, x0, tg = _sim(ddm, "f32", [th[i]])
        sim.set_grad_treatment("norm", record_steps=STEPS)
        g = _grad(sim, x0, tg)
        S = sim.grad_stats()
        _log(f"instance {i}: batched {gb[i]} alone {g[0]}")
        _same(gb[i], g[0], "f32", f"gradient of instance {i}")
        _same_record(Sb[:, i], S[:, 0], "f32", f"record of instance {i}")


def test_graph_pass_with_treatment(ddm):
    import torch
    _log("case treat scale graph pass f32")
    w, _, x0, tg = _sim(ddm, "f32")
    cfg, inst = ddm.from_workload(w, max_steps=STEPS, checkpoint_every=16, precision="f32")
    stream = torch.cuda.Stream()
    sim = ddm.Simulator(cfg, [inst], stream=stream)
    sim.set_grad_treatment("none", record_steps=STEPS)
    _grad(sim, x0, tg)
    c, oom = _acting_thresholds(sim.grad_stats())
    sim.set_grad_treatment("scale", oom=oom, record_steps=STEPS)
    ge = _grad(sim, x0, tg)
    Se = sim.grad_stats()
    for rep in range(3):
        loss, grad = sim.full_pass(x0, STEPS, tg, graph=True)
        torch.cuda.synchronize()
        g = grad.cpu().numpy()
        _log(f"replay {rep}: {g[0]}")
        _same(g, ge, "f32", f"gradient of replay {rep}")
        _same_record(sim.grad_stats(), Se, "f32", f"record of replay {rep}")


def test_optimiser_evaluator_applies_treatment(ddm):
    """GpuEvaluator(treatment=...) computes its gradients with the treatment."""
    from paper_2510_17335_amd import optim as O
    _log("case evaluator with clip f32")
    w = W.dig_3d(steps=STEPS)
    x0, tg = W.bed_positions(w), W.target_heightmap(w)
    plain = O.GpuEvaluator(ddm, w, x0, tg, STEPS, batch=2, checkpoint_every=16, precision="f32")
    _, g0 = plain.grad(w.params)
    _, sim, xs, tgs = _sim(ddm, "f32")
    sim.set_grad_treatment("none", record_steps=STEPS)
    _grad(sim, xs, tgs)
    c, _ = _acting_thresholds(sim.grad_stats())
    sim.set_grad_treatment("clip", clip=c)
    gs = _grad(sim, xs, tgs)[0]
    ev = O.GpuEvaluator(ddm, w, x0, tg, STEPS, batch=2, checkpoint_every=16, precision="f32",
                        treatment={"mode": "clip", "clip": c})
    _, g1 = ev.grad(w.params)
    _same(g1, gs, "f32", "evaluator with clip")
    assert not np.allclose(g1, g0, rtol=1e-3)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("mode", ["none", "clip", "scale", "norm"])
def test_treated_gradient_matches_reverse_oracle(ddm, orc, dim, mode):
    """Element-wise reference for the treatments: the FP64 GPU pass against
    the oracle's reverse-mode tape (its untreated gradient is pinned to the
    forward-mode one), which treats the same vectors at the same points of
    its adjoint sweep.  Tiny beds; the recorded rollout (40 sub-steps, K = 16)
    starts after 20 untreated sub-steps, so that no particle sits at F = I,
    the apex of the return map, where round-off picks the case.  Thresholds
    act on about half of the vectors.  The 9 parameter gradients agree to
    1e-8."""
    pre, steps = 20, 40
    w = W.tiny(dim, shovel=(dim == 3), steps=pre + steps)
    w.precision = "f64"
    if w.target_seed is None:
        w.target_seed = 11
    x0, tg = W.bed_positions(w), W.target_heightmap(w)
    cfg = orc.config(w)
    s20 = orc.rollout(cfg, w.params, orc.initial_state(x0), pre)["state"]
    r0 = orc.rollout_reverse(cfg, w.params, s20, steps, tg, step0=pre, stats=True)
    c, oom = _acting_thresholds(r0["stats"][:, None])
    ref = orc.rollout_reverse(cfg, w.params, s20, steps, tg, step0=pre, mode=mode, clip=c, oom=oom, delta=1e-6,
                              stats=True)
    _log(f"case treated gradient vs reverse oracle dim {dim} {mode} (clip {c}, oom* {oom})")
    dcfg, inst = ddm.from_workload(w, max_steps=pre + steps, checkpoint_every=16)
    sim = ddm.Simulator(dcfg, [inst])
    sim.set_grad_treatment(mode, clip=c, oom=oom, delta=1e-6, record_steps=pre + steps)
    sim.init_state(x0)
    sim.step(pre)
    sim.rollout(steps)
    loss = float(sim.loss(tg[None])[0])
    g = sim.backward()[0].cpu().numpy()
    assert sim.check().flags & 1 == 0
    rg = ref["grad"]
    scale = np.abs(rg).max()
    rel = np.abs(g - rg) / np.maximum(np.abs(rg), 1e-9 * scale)
    acted = int(np.sum(np.any(ref["stats"][..., :3] != ref["stats"][..., 3:], axis=-1)))
    _log(f"loss {loss} vs {ref['loss']}; {acted} of {steps * 6} vectors treated\ngpu {g}\noracle {rg}\nrel {rel}")
    assert abs(loss - ref["loss"]) <= 1e-12 * abs(ref["loss"])
    if mode != "none":
        assert acted > 0 and not np.allclose(rg, r0["grad"], rtol=1e-6)
    assert np.all(rel < 1e-8), rel
    # every adjoint vector, before and after its treatment: max, min and 2-norm
    # within 1e-9 of that vector's norm (the same elements on both sides)
    S, R = sim.grad_stats()[pre:, 0], ref["stats"]
    for post in (0, 3):
        ref_norm = np.maximum(R[..., post + 2:post + 3], 1e-300)
        err = np.abs(S[..., post:post + 3] - R[..., post:post + 3]) / ref_norm
        assert np.all(err < 1e-9), (post, np.unravel_index(np.argmax(err), err.shape), err.max())
