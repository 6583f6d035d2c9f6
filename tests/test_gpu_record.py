"""Recording the last checkpoint segments during the rollout
(ddm_config.record_segments) changes where the reverse pass finds the data of
each sub-step, not what it computes: final states, losses and gradients agree
with 1, 2 and all segments recorded as closely as two runs of one setting do
(the order of atomic sums varies), also for a second reverse pass after the
first, which replays every segment from its checkpoint; the
workspace grows by one segment set per recorded segment, up to the segments
of a max_steps rollout.  A record of the pre-update grids that holds only
the active blocks (ddm_config.grid_record_blocks) gives the same pass while
it is large enough, and flags DDM_ENOMEM when it is not."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

STEPS, K = 60, 16          # four segments, the last one of 12 sub-steps


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ddm():
    import torch
    assert torch.cuda.is_available()
    import paper_2510_17335_amd as m
    return m


def _run(ddm, record, precision="f32", passes=1, grid_blocks=0, check=True):
    w = W.dig_3d(steps=STEPS)
    cfg, inst = ddm.from_workload(w, max_steps=STEPS, checkpoint_every=K, precision=precision)
    cfg.record_segments = record
    cfg.grid_record_blocks = grid_blocks
    sim = ddm.Simulator(cfg, [inst])
    x0, tg = W.bed_positions(w), W.target_heightmap(w).reshape(1, -1)
    sim.init_state(x0)
    sim.rollout(STEPS)
    state = sim.packed_state(0)            # decoded: x, v, C, F per particle
    loss = sim.loss(tg).cpu().numpy()
    grads = [sim.backward().cpu().numpy() for _ in range(passes)]
    if check:
        assert sim.check().flags & 1 == 0
        return int(sim.sizes.workspace_bytes), state, loss, grads
    return sim


def _close(a, b, what, rtol=1e-6):
    rel = float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-30)))
    _log(f"{what}: max relative difference {rel:.3e}")
    assert rel <= rtol, (what, a, b)


def _same_state(a, b, what, rtol):
    """Per state component (x, v, C, F entries) the largest difference
    relative to the component's largest magnitude."""
    rel = np.max(np.abs(a - b), axis=0) / np.maximum(np.max(np.abs(b), axis=0), 1e-30)
    _log(f"{what}: largest relative state difference {float(rel.max()):.3e} (component {int(rel.argmax())})")
    assert float(rel.max()) <= rtol, what


def test_recorded_segments_give_the_same_pass(ddm):
    _log(f"case record_segments 1/2/4/9 dig3d {STEPS} steps K={K} f32")
    ws1, s1, l1, g1 = _run(ddm, 1, passes=2)
    _close(g1[1], g1[0], "second reverse pass, every segment replayed")
    ws0, s0, l0, g0 = _run(ddm, 0)
    assert ws0 == ws1
    # run to run: particles that drift out of their tile's window add to the
    # grid with FP32 atomics, whose order varies
    _same_state(s0, s1, "same setting, second run", 1e-5)
    prev = ws1
    for r in (2, 4):
        ws, s, l, g = _run(ddm, r)
        _log(f"record_segments {r}: workspace {ws / 2**30:.2f} GiB (1: {ws1 / 2**30:.2f} GiB)")
        assert ws > prev
        prev = ws
        _same_state(s, s1, f"final state with {r} segments recorded", 1e-5)
        _close(l, l1, "loss", rtol=1e-6)
        _close(g[0], g1[0], f"gradient with {r} segments recorded", rtol=1e-5)
    # more sets than segments: capped
    assert _run(ddm, 9)[0] == prev


def test_recorded_segments_f64(ddm):
    _log(f"case record_segments 1/4 dig3d {STEPS} steps K={K} f64")
    _, s1, l1, g1 = _run(ddm, 1, precision="f64")
    _, s4, l4, g4 = _run(ddm, 4, precision="f64")
    # FP64 sums add in a different order from run to run (about 1e-15 of the state)
    _close(l4, l1, "loss", rtol=1e-10)
    _close(g4[0], g1[0], "gradient", rtol=1e-8)


def test_graph_replays_with_recorded_segments(ddm):
    """A pass captured into a HIP graph with two segments recorded gives the
    eager gradient on every replay, with eager work between the replays."""
    import torch
    _log(f"case record_segments 2 graph replays dig3d {STEPS} steps K={K} f32")
    w = W.dig_3d(steps=STEPS)
    cfg, inst = ddm.from_workload(w, max_steps=STEPS, checkpoint_every=K, precision="f32")
    cfg.record_segments = 2
    sim = ddm.Simulator(cfg, [inst], stream=torch.cuda.Stream())
    x0, tg = W.bed_positions(w), W.target_heightmap(w).reshape(1, -1)
    sim.init_state(x0)
    sim.rollout(STEPS)
    l_e = sim.loss(tg).cpu().numpy()
    g_e = sim.backward().cpu().numpy()
    for rep in range(3):
        loss, grad = sim.full_pass(x0, STEPS, tg, graph=True)
        torch.cuda.synchronize()
        _close(loss.cpu().numpy(), l_e, f"loss of replay {rep}", rtol=1e-6)
        _close(grad.cpu().numpy(), g_e, f"gradient of replay {rep}", rtol=1e-5)
        # eager work of the program between replays
        sim.init_state(x0)
        sim.step(3)
        torch.cuda.synchronize()
    assert sim.check().flags & 1 == 0


def test_autotune_between_rollout_and_backward(ddm):
    """ddm_autotune probes from the current state in the segment buffers: a
    reverse pass after it replays every segment from its snapshot and gives
    the gradient of an undisturbed pass."""
    _log(f"case autotune after a rollout with all segments recorded, dig3d {STEPS} steps K={K} f32")
    _, _, _, g1 = _run(ddm, 1)
    w = W.dig_3d(steps=STEPS)
    cfg, inst = ddm.from_workload(w, max_steps=STEPS, checkpoint_every=K, precision="f32")
    cfg.record_segments = 4
    sim = ddm.Simulator(cfg, [inst])
    x0, tg = W.bed_positions(w), W.target_heightmap(w).reshape(1, -1)
    sim.init_state(x0)
    sim.rollout(STEPS)
    sim.loss(tg)
    sim.autotune()
    g = sim.backward().cpu().numpy()
    assert sim.check().flags & 1 == 0
    _close(g, g1[0], "gradient after autotune", rtol=1e-5)


def _active_blocks(ddm, precision):
    """The most active blocks over the sub-steps of a forward run of the dig."""
    w = W.dig_3d(steps=STEPS)
    cfg, inst = ddm.from_workload(w, max_steps=STEPS, checkpoint_every=K, precision=precision)
    sim = ddm.Simulator(cfg, [inst])
    sim.init_state(W.bed_positions(w))
    most = 0
    for _ in range(STEPS):
        sim.step(1)
        g = sim.get_grid()
        most = max(most, int(round(float((g[0, :, 7] > 0).sum().item()) / 64)))
    return most


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_grid_record_of_active_blocks(ddm, precision):
    """The pre-update grids recorded as their active blocks only, with the
    capacity set to the most active blocks of the run (every sub-step fits,
    the largest exactly): the same final state, loss and gradient as the full
    record, for all segments recorded (4) and for one (the others replayed
    into the same smaller buffers); the workspace shrinks."""
    most = _active_blocks(ddm, precision)
    _log(f"case grid record of {most} active blocks (of 4096), dig3d {STEPS} steps K={K} {precision}")
    assert 0 < most < 4096
    tol = (1e-10, 1e-8) if precision == "f64" else (1e-6, 1e-5)
    for record in (4, 1):
        wsf, sf, lf, gf = _run(ddm, record, precision=precision)
        wsc, sc, lc, gc = _run(ddm, record, precision=precision, grid_blocks=most)
        _log(f"record_segments {record}: workspace {wsc / 2**30:.3f} GiB against {wsf / 2**30:.3f} GiB")
        assert wsc < wsf
        _same_state(sc, sf, f"final state, {record} recorded", 1e-5 if precision == "f32" else 1e-12)
        _close(lc, lf, "loss", rtol=tol[0])
        _close(gc[0], gf[0], f"gradient, {record} recorded", rtol=tol[1])


def test_grid_record_too_small_is_flagged(ddm):
    """A capacity below what a recorded sub-step needs: the grid update writes
    only what fits, the reverse pass reads the rest as empty nodes, and
    ddm_check reports DDM_ENOMEM with device error bit 4."""
    _log(f"case grid record of 8 blocks, dig3d {STEPS} steps K={K} f32")
    sim = _run(ddm, 2, grid_blocks=8, check=False)
    with pytest.raises(ddm.DdmError) as e:
        sim.check()
    assert e.value.code == ddm.DDM_ENOMEM
    err = ddm.DdmDeviceError()
    ddm.lib().ddm_check(sim.ctx, ddm.C.byref(err))
    assert err.flags & 16
