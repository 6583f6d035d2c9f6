"""The deterministic mode (ddm_config.deterministic) through the C-ABI.

* Bitwise equality of the final state, the loss and the gradient between two
  runs, between launch shapes (one workgroup per tile against a persistent
  launch of 8 workgroups, which hands the tiles to other workgroups in
  another order), and between a pass that replays its checkpoint segments and
  one that records them all; on the tiny 3D bed with the shovel and the
  particle-level collision (every reduction of the pass: the P2G and G2P
  adjoint windows, the material, density and pose adjoints, the scoop mass),
  in FP64 and FP32, and on an 8-instance FP32 batch of the system
  identification workload.
* The deterministic sums are a reordering of the default mode's: FP64
  results agree with the default mode and with the oracle to round-off.
* A state taken mid-run and set into another context continues bitwise to
  the uninterrupted run's state (a cell's particles are ordered by id at
  every binning, whatever their order before).
* The normalisation treatment, whose 2-norm is reduced with atomics, is
  rejected.
"""
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


def _tiny(precision):
    w = W.tiny(3, shovel=True, steps=40)
    w.precision = precision
    w.particle_contact = True
    return w


def _pass(ddm, ws, steps, det=True, workgroups=0, record_segments=1, K=16):
    cfgs = [ddm.from_workload(w, max_steps=steps, checkpoint_every=K, deterministic=det) for w in ws]
    cfg = cfgs[0][0]
    cfg.tile_workgroups = workgroups
    cfg.record_segments = record_segments
    sim = ddm.Simulator(cfg, [c[1] for c in cfgs])
    sim.init_state(np.concatenate([W.bed_positions(w) for w in ws]))
    sim.rollout(steps)
    loss = sim.loss(np.stack([W.target_heightmap(w) for w in ws])).cpu().numpy()
    grad = sim.backward().cpu().numpy()
    err = sim.check()
    assert err.flags == 0 and err.clamp_count == 0, err.flags
    state = np.concatenate([sim.packed_state(i) for i in range(len(ws))])
    return state, loss, grad


def _same(a, b, what):
    for x, y, name in zip(a, b, ("state", "loss", "gradient")):
        if not np.array_equal(x, y):
            d = np.abs(x - y).max()
            raise AssertionError(f"{what}: {name} differs (largest difference {d:.3e})")


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_bitwise_across_runs_launches_and_replays(ddm, precision):
    w = _tiny(precision)
    _log(f"case deterministic tiny3d {precision}: two runs, 8 persistent workgroups, all segments recorded")
    ref = _pass(ddm, [w], 40)
    _same(ref, _pass(ddm, [w], 40), "second run")
    _same(ref, _pass(ddm, [w], 40, workgroups=8), "8 persistent workgroups")
    _same(ref, _pass(ddm, [w], 40, record_segments=3), "all segments recorded")
    assert np.all(np.isfinite(ref[2])) and np.abs(ref[2]).max() > 0


def test_close_to_default_mode_and_oracle_f64(ddm, orc):
    w = _tiny("f64")
    det = _pass(ddm, [w], 40)
    dflt = _pass(ddm, [w], 40, det=False)
    scale = np.abs(dflt[0]).max(axis=0)
    ds = (np.abs(det[0] - dflt[0]).max(axis=0) / np.maximum(scale, 1e-30)).max()
    rel = np.abs(det[2] - dflt[2]) / np.maximum(np.abs(dflt[2]), 1e-9 * np.abs(dflt[2]).max())
    _log(f"deterministic vs default FP64: state {ds:.2e}, loss {abs(det[1][0] - dflt[1][0]):.2e}, grad {rel.max():.2e}")
    assert ds < 1e-12
    assert abs(det[1][0] - dflt[1][0]) <= 1e-12 * abs(dflt[1][0])
    assert np.all(rel < 1e-9), rel
    ocfg = orc.config(w)
    r = orc.rollout(ocfg, w.params, orc.initial_state(W.bed_positions(w)), 40, target=W.target_heightmap(w),
                    grad=True)
    orel = np.abs(det[2][0] - r["grad"]) / np.maximum(np.abs(r["grad"]), 1e-9 * np.abs(r["grad"]).max())
    _log(f"deterministic FP64 vs oracle: loss {det[1][0]!r} vs {r['loss']!r}, grad {orel.max():.2e}")
    assert abs(det[1][0] - r["loss"]) <= 1e-10 * abs(r["loss"])
    assert np.all(orel < 1e-6), orel


def test_batch_bitwise_across_launches_f32(ddm):
    ws = W.sysid_batch(8, steps=30)
    _log("case deterministic sysid batch of 8, FP32, 30 sub-steps: one workgroup per tile vs 1024 persistent")
    a = _pass(ddm, ws, 30, K=10)
    b = _pass(ddm, ws, 30, K=10, workgroups=1024)
    _same(a, b, "1024 persistent workgroups")


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_resume_is_bitwise(ddm, precision):
    w = W.dig_3d(steps=40)
    w.precision = precision
    cfg, inst = ddm.from_workload(w, max_steps=40, checkpoint_every=20, deterministic=True)
    x0 = W.bed_positions(w)
    _log(f"case deterministic resume, 64^3 dig {precision}")
    a = ddm.Simulator(cfg, [inst])
    a.init_state(x0)
    a.step(20)
    saved = a.get_state()
    a.step(20)
    b = ddm.Simulator(cfg, [inst])
    b.init_state(x0)
    b.step(20)
    b.set_state(saved)
    b.step(20)
    assert a.check().flags == 0 and b.check().flags == 0
    assert np.array_equal(a.packed_state(0), b.packed_state(0))


def test_normalisation_rejected(ddm):
    w = _tiny("f64")
    cfg, inst = ddm.from_workload(w, max_steps=40, checkpoint_every=16, deterministic=True)
    sim = ddm.Simulator(cfg, [inst])
    with pytest.raises(ddm.DdmError):
        sim.set_grad_treatment("norm")
    sim.set_grad_treatment("clip")
    sim.set_grad_treatment("scale")
