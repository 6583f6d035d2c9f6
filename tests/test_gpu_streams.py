"""A batch run as several contexts at once (StreamGroup): the groups'
passes, issued on their own streams without waits between them and replayed
from captured graphs, give the losses and gradients of one context over the
whole batch, in the original instance order (FP64, so the only difference is
the order of atomic sums); in the deterministic mode, bit for bit."""
import sys
from dataclasses import replace

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


def _batch():
    base = W.tiny(3, shovel=True, steps=24)
    beds = [((6, 3, 6), (10, 5, 8)), ((5, 3, 5), (11, 5, 10)), ((6, 3, 6), (8, 5, 8)), ((5, 3, 6), (10, 6, 9))]
    ws = []
    for k, (lo, hi) in enumerate(beds):
        ws.append(replace(base, bed_lo=lo, bed_hi=hi, seed=base.seed + k))
    return ws


@pytest.mark.parametrize("graph", [True, False])
def test_stream_group_equals_one_context(ddm, graph):
    import torch
    ws = _batch()
    cfgs = [ddm.from_workload(w, max_steps=24, checkpoint_every=8) for w in ws]
    cfg, insts = cfgs[0][0], [c[1] for c in cfgs]
    for k, q in enumerate(insts):
        q.E *= 1.0 + 0.2 * k                     # a different modulus per instance
    x0 = np.concatenate([W.bed_positions(w) for w in ws])
    tg = np.stack([W.target_heightmap(w) for w in ws])
    one = ddm.Simulator(cfg, insts, stream=torch.cuda.Stream())
    l1, g1 = one.full_pass(x0, 24, tg)
    l1, g1 = l1.cpu().numpy(), g1.cpu().numpy()
    groups = ddm.balanced_groups([w.n_particles for w in ws], 2)
    _log(f"case stream group {groups}, graph={graph}, particles {[w.n_particles for w in ws]}")
    sg = ddm.StreamGroup(cfg, insts, groups)
    for rep in range(3):
        ls, gs = sg.full_pass(torch.as_tensor(x0, device="cuda"), 24, tg, graph=graph)
        ls, gs = ls.cpu().numpy(), gs.cpu().numpy()
        assert sg.check().flags == 0
        rel = np.abs(gs - g1) / np.maximum(np.abs(g1), 1e-9 * np.abs(g1).max())
        _log(f"pass {rep}: loss {np.abs(ls - l1).max():.2e}, grad rel {rel.max():.2e}")
        np.testing.assert_allclose(ls, l1, rtol=1e-12)
        assert np.all(rel < 1e-9), rel


def test_unjoined_runs_keep_the_last_results(ddm):
    """Passes issued back to back with run(), each group queued behind its
    own previous pass only, and passes joined by join() after each run():
    results() gives the last pass's losses and gradients, those of a joined
    full_pass."""
    import torch
    ws = _batch()
    cfgs = [ddm.from_workload(w, max_steps=24, checkpoint_every=8) for w in ws]
    cfg, insts = cfgs[0][0], [c[1] for c in cfgs]
    x0 = np.concatenate([W.bed_positions(w) for w in ws])
    tg = np.stack([W.target_heightmap(w) for w in ws])
    sg = ddm.StreamGroup(cfg, insts, ddm.balanced_groups([w.n_particles for w in ws], 3))
    _log(f"case stream group of 3, three unjoined graph-replayed runs, groups {sg.groups}")
    l1, g1 = (a.cpu().numpy() for a in sg.full_pass(x0, 24, tg))
    sg.set_inputs(x0, tg)
    for _ in range(3):
        sg.run(24)
    ls, gs = (a.cpu().numpy() for a in sg.results())
    assert sg.check().flags == 0
    rel = np.abs(gs - g1) / np.maximum(np.abs(g1), 1e-9 * np.abs(g1).max())
    np.testing.assert_allclose(ls, l1, rtol=1e-12)
    assert np.all(rel < 1e-9), rel
    # joined steps: run, then the current stream waits for every group
    for _ in range(2):
        sg.run(24)
        sg.join()
    ls, gs = (a.cpu().numpy() for a in sg.results())
    rel = np.abs(gs - g1) / np.maximum(np.abs(g1), 1e-9 * np.abs(g1).max())
    np.testing.assert_allclose(ls, l1, rtol=1e-12)
    assert np.all(rel < 1e-9), rel


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_deterministic_groups_are_bitwise_one_context(ddm, precision):
    """In the deterministic mode an instance's sums do not depend on the
    other instances of its batch (fixed-order window passes, per-instance
    partials summed in a fixed order), so two concurrent groups give the
    single context's losses and gradients bit for bit."""
    import torch
    ws = _batch()
    for w in ws:
        w.precision = precision
    cfgs = [ddm.from_workload(w, max_steps=24, checkpoint_every=8, deterministic=True) for w in ws]
    cfg, insts = cfgs[0][0], [c[1] for c in cfgs]
    x0 = np.concatenate([W.bed_positions(w) for w in ws])
    tg = np.stack([W.target_heightmap(w) for w in ws])
    one = ddm.Simulator(cfg, insts, stream=torch.cuda.Stream())
    l1, g1 = (a.cpu().numpy() for a in one.full_pass(x0, 24, tg))
    sg = ddm.StreamGroup(cfg, insts, ddm.balanced_groups([w.n_particles for w in ws], 2))
    _log(f"case deterministic stream group {sg.groups}, {precision}")
    ls, gs = (a.cpu().numpy() for a in sg.full_pass(x0, 24, tg))
    assert sg.check().flags == 0 and one.check().flags == 0
    assert np.array_equal(ls, l1), np.abs(ls - l1).max()
    assert np.array_equal(gs, g1), np.abs(gs - g1).max()
