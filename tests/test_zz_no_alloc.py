"""ddm_loss_noalloc, the entry point that allocates nothing (its scratch is a
static device array), against ddm_loss through a context: the loss and the
height map of the same positions, two calls in a row, the second with fewer
particles; in FP64 with positions taken from a context after 30 sub-steps
(the blade at that sub-step's pose) and in FP32 with the initial positions
(the initial pose).  Height maps agree exactly; the loss to 1e-12 (its
scoop mass is a sum of FP64 atomics, whose order may differ).  Also the
argument checks."""
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


def _context_loss(ddm, w, steps):
    """Loss, height map and positions (context precision) after `steps` sub-steps."""
    import torch
    x0 = W.bed_positions(w)
    target = W.target_heightmap(w)
    cfg, inst = ddm.from_workload(w, max_steps=max(steps, 1))
    sim = ddm.Simulator(cfg, [inst])
    sim.init_state(x0)
    if steps:
        sim.step(steps)
    loss = sim.loss(target[None])[0].item()
    hm = sim.heightmap()[0].cpu().numpy()
    if steps:    # FP64: the state holds the positions as doubles
        x = torch.as_tensor(sim.packed_state(0)[:, :w.dim], dtype=sim.dtype, device="cuda")
    else:
        x = torch.as_tensor(x0, dtype=sim.dtype, device="cuda")
    return cfg, inst, target, loss, hm, x


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_noalloc_loss_equals_context_loss_twice(ddm, prec):
    import torch
    steps = 30 if prec == "f64" else 0
    for call, ppc in enumerate([8, 1]):
        w = W.dig_3d(steps=max(steps, 1), ppc=ppc)
        w.precision = prec
        cfg, inst, target, ref, ref_hm, x = _context_loss(ddm, w, steps)
        print(f"case noalloc {prec} call {call + 1}: {x.shape[0]} particles, blade after sub-step {steps - 1}",
              flush=True)
        loss, hm = ddm.loss_noalloc(cfg, inst, steps - 1, x, target)
        torch.cuda.synchronize()
        got, got_hm = loss.item(), hm.cpu().numpy()
        print(f"  context {ref!r}  no-alloc {got!r}", flush=True)
        assert abs(got - ref) <= 1e-12 * abs(ref)
        assert np.array_equal(got_hm, ref_hm)


def test_noalloc_rejects_what_does_not_fit(ddm):
    import torch
    w = W.dig_3d(steps=4)
    cfg, inst = ddm.from_workload(w, max_steps=4)
    x = torch.zeros((10, 3), dtype=torch.float32, device="cuda")
    tg = W.target_heightmap(w)
    inst.n_particles = 262145
    with pytest.raises(ddm.DdmError, match="DDM_NOALLOC_MAX_PARTICLES"):
        ddm.loss_noalloc(cfg, inst, 0, x, tg)
    inst.n_particles = 10
    with pytest.raises(ddm.DdmError, match="final_step"):
        ddm.loss_noalloc(cfg, inst, 4, x, tg)
    cfg.hm_res = 65
    with pytest.raises(ddm.DdmError, match="DDM_NOALLOC_MAX_PIXELS"):
        ddm.loss_noalloc(cfg, inst, 0, x, np.zeros(65 * 65))
