"""ddm_diagnostics through the C-ABI against the oracle's diagnostics of the
same state: FP64 tiny beds (2D, and 3D with the blade) after 20 sub-steps,
with sums to round-off, return-map case counts exact, the CFL number, and
the grid mass of the last sub-step against the oracle's grid; the 64^3 dig
in FP32 (sums to 1e-5, case counts within 0.5 % of N); a NaN grid mass when
there is no grid; and resuming: a state taken mid-run and set into another
context continues to the final state and diagnostics of the uninterrupted
run (FP64 to round-off)."""
import math
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


def _compare(gd, od, grid_mass, rel_sum, case_tol):
    names = ("mass", "px", "py", "pz", "ke", "tension", "elastic", "projected", "clamps", "cfl", "grid mass")
    _log("gpu   ", dict(zip(names, np.round(gd, 12))))
    _log("oracle", dict(zip(names, np.round(od, 12))), "grid mass", grid_mass)
    assert gd[0] == pytest.approx(od[0], rel=rel_sum)
    scale = max(abs(od[1:4]).max(), 1e-30)
    np.testing.assert_allclose(gd[1:4], od[1:4], rtol=0, atol=rel_sum * 10 * scale)
    assert gd[4] == pytest.approx(od[4], rel=rel_sum * 10)
    assert np.all(np.abs(gd[5:8] - od[5:8]) <= case_tol), (gd[5:8], od[5:8])
    assert gd[8] == od[8] == 0
    assert gd[9] == pytest.approx(od[9], rel=rel_sum * 10)
    assert gd[10] == pytest.approx(grid_mass, rel=rel_sum)


@pytest.mark.parametrize("d", [2, 3])
def test_diagnostics_match_oracle_f64(ddm, orc, d):
    steps = 20
    w = W.tiny(d, shovel=(d == 3), steps=steps)
    w.precision = "f64"
    cfg, inst = ddm.from_workload(w, max_steps=steps, checkpoint_every=steps)
    sim = ddm.Simulator(cfg, [inst])
    x0 = W.bed_positions(w)
    sim.init_state(x0)
    g0 = sim.diagnostics()[0]
    assert math.isnan(g0[10])
    _log(f"case diagnostics tiny{d}d f64 after {steps} sub-steps")
    sim.step(steps)
    gd = sim.diagnostics()[0]
    assert sim.check().flags == 0
    ocfg = orc.config(w)
    r = orc.rollout(ocfg, w.params, orc.initial_state(x0), steps, want_grid=True)
    od = orc.diagnostics(ocfg, w.params, r["state"])
    assert od[5:8].sum() == w.n_particles
    _compare(gd, od, r["grid"][:, 0].sum(), 1e-11, 0)


def test_diagnostics_dig3d_f32(ddm, orc):
    steps = 60
    w = W.dig_3d(steps=steps)
    cfg, inst = ddm.from_workload(w, max_steps=steps, checkpoint_every=20)
    sim = ddm.Simulator(cfg, [inst])
    x0 = W.bed_positions(w)
    sim.init_state(x0)
    _log(f"case diagnostics dig3d f32 after {steps} sub-steps")
    sim.step(steps)
    gd = sim.diagnostics()[0]
    err = sim.check()
    assert err.flags == 0 and err.clamp_count == 0
    ocfg = orc.config(w)
    r = orc.rollout(ocfg, w.params, orc.initial_state(x0), steps)
    od = orc.diagnostics(ocfg, w.params, r["state"])
    # FP32 states: sums to about 1e-5, cases of particles near a case boundary may differ
    _compare(gd, od, od[0], 1e-5, 0.005 * w.n_particles)


def test_no_grid_after_backward(ddm):
    steps = 12
    w = W.tiny(3, shovel=True, steps=steps)
    cfg, inst = ddm.from_workload(w, max_steps=steps, checkpoint_every=6)
    sim = ddm.Simulator(cfg, [inst])
    sim.init_state(W.bed_positions(w))
    sim.rollout(steps)
    after_rollout = sim.diagnostics()[0]
    # the rollout's last grid is rebuilt from its record: it holds the particle mass
    assert after_rollout[10] == pytest.approx(after_rollout[0], rel=1e-5)
    sim.loss(W.target_heightmap(w)[None])
    sim.backward()
    assert math.isnan(sim.diagnostics()[0][10])


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_resume_from_a_saved_state(ddm, precision):
    """Binning every 20 sub-steps; the state after 20 of 40 sub-steps, set into
    a second context that has taken 20 sub-steps of its own (so that the blade
    pose follows the same step count), continues to the state and
    diagnostics of the uninterrupted run.  After ddm_set_state the particle
    ids restart, so particles of one cell are summed in another order: FP64
    agrees to round-off; in FP32 the states agree to about 1e-6, and a
    particle that the previous sub-step projected onto the yield surface can
    take the other side of it (about 0.05 % of the particles)."""
    w = W.dig_3d(steps=40)
    w.precision = precision
    cfg, inst = ddm.from_workload(w, max_steps=40, checkpoint_every=20, sort_every=20)
    x0 = W.bed_positions(w)
    a = ddm.Simulator(cfg, [inst])
    a.init_state(x0)
    a.step(20)
    saved = a.get_state()
    a.step(20)
    ref, dref = a.packed_state(0), a.diagnostics()[0]
    b = ddm.Simulator(cfg, [inst])
    b.init_state(x0)
    b.step(20)
    b.set_state(saved)
    b.step(20)
    got, dgot = b.packed_state(0), b.diagnostics()[0]
    assert a.check().flags == 0 and b.check().flags == 0
    diff = np.abs(got - ref).max(axis=0) / np.maximum(np.abs(ref).max(axis=0), 1e-30)
    _log(f"resumed against uninterrupted ({precision}): largest relative state difference {diff.max():.3e}; "
         f"case counts {dgot[5:8]} against {dref[5:8]}")
    tol = {"f64": (1e-12, 1e-12, 0.0002), "f32": (1e-5, 1e-5, 0.005)}[precision]
    assert diff.max() <= tol[0]
    np.testing.assert_allclose(dgot[:5], dref[:5], rtol=tol[1], atol=1e-12)
    assert np.all(np.abs(dgot[5:8] - dref[5:8]) <= tol[2] * w.n_particles)
