"""DigLoss, the torch.autograd.Function over the library's rollout, loss and
reverse pass (the gradient chain of Eq. grad-chain), on the tiny 3D dig in
FP64: torch.autograd.grad through dig_loss equals Simulator.backward and the
oracle's forward-mode gradient, for parameters held on the CPU and on the
GPU, with an upstream gradient that is not all ones."""
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


def _case(seed):
    w = W.tiny(3, shovel=True, steps=40, seed=seed)
    w.precision = "f64"
    return w


@pytest.mark.parametrize("param_device", ["cpu", "cuda"])
def test_dig_loss_autograd_matches_backward_and_oracle(ddm, orc, param_device):
    import torch
    ws = [_case(7), _case(8)]
    ws[1].material.E = 2.0e5
    ws[1].skill.angle_deg = 25.0
    print(f"case DigLoss tiny3d x2 f64, params on {param_device}", flush=True)
    cfgs = [ddm.from_workload(w, max_steps=w.steps, checkpoint_every=10) for w in ws]
    cfg, insts = cfgs[0][0], [c[1] for c in cfgs]
    x0 = torch.tensor(np.concatenate([W.bed_positions(w) for w in ws]), device="cuda")
    tg = torch.tensor(np.stack([W.target_heightmap(w) for w in ws]), device="cuda")
    params = torch.tensor(np.stack([w.params for w in ws]), dtype=torch.float64, device=param_device,
                          requires_grad=True)
    loss = ddm.dig_loss(params, x0, tg, cfg, insts, ws[0].steps)
    assert loss.device == params.device and loss.shape == (2,)
    up = torch.tensor([2.5, -0.75], dtype=torch.float64, device=param_device)
    (g,) = torch.autograd.grad((loss * up).sum(), params)
    assert g.device == params.device and g.dtype == torch.float64 and g.shape == params.shape
    g = g.cpu().numpy()

    sim = ddm.Simulator(cfg, insts)
    sim.init_state(x0)
    sim.rollout(ws[0].steps)
    l2 = sim.loss(tg).cpu().numpy()
    gb = sim.backward().cpu().numpy()
    np.testing.assert_allclose(loss.detach().cpu().numpy(), l2, rtol=1e-12)
    upn = up.cpu().numpy()
    np.testing.assert_allclose(g, gb * upn[:, None], rtol=1e-9, atol=1e-12 * np.abs(g).max())

    for i, w in enumerate(ws):
        r = orc.rollout(orc.config(w), w.params, orc.initial_state(W.bed_positions(w)), w.steps,
                        target=W.target_heightmap(w), grad=True)
        assert abs(l2[i] - r["loss"]) <= 1e-9 * abs(r["loss"])
        ref = r["grad"] * upn[i]
        rel = np.abs(g[i] - ref) / np.maximum(np.abs(ref), 1e-9 * np.abs(ref).max())
        print(f"instance {i}: DigLoss gradient vs oracle, max rel err {rel.max():.2e}", flush=True)
        assert np.all(rel < 1e-6), rel


def test_dig_loss_second_backward_and_f32_params(ddm, orc):
    """A float32 parameter tensor gets a float32 gradient; a retained graph
    can run its backward twice (the second call replays every segment)."""
    import torch
    w = _case(7)
    cfg, inst = ddm.from_workload(w, max_steps=w.steps, checkpoint_every=10)
    x0 = W.bed_positions(w)
    tg = W.target_heightmap(w)[None]
    params = torch.tensor(w.params[None], dtype=torch.float32, requires_grad=True)
    loss = ddm.dig_loss(params, x0, tg, cfg, [inst], w.steps)
    loss.sum().backward(retain_graph=True)
    g1 = params.grad.clone()
    params.grad = None
    loss.sum().backward()
    assert params.grad.dtype == torch.float32
    np.testing.assert_allclose(params.grad.numpy(), g1.numpy(), rtol=1e-6)
