"""Kernel timing through the C-ABI: a group mask brackets only the selected
launch groups with events, every group when all are selected, and a mask
outside the defined groups is rejected."""
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


def test_timing_groups(ddm):
    w = W.tiny(3, shovel=True, steps=12)
    cfg, inst = ddm.from_workload(w, max_steps=12, checkpoint_every=4)
    sim = ddm.Simulator(cfg, [inst])
    sim.init_state(W.bed_positions(w))
    sim.set_timing(groups=["p2g"])
    sim.step(4)
    t = sim.read_timing()
    assert t["p2g"][1] == 4 and t["p2g"][0] > 0
    assert all(n == 0 for k, (ms, n) in t.items() if k != "p2g"), t
    sim.set_timing(True)
    sim.step(4)
    t = sim.read_timing()
    assert t["p2g"][1] == 4 and t["grid_update"][1] == 4 and t["g2p"][1] == 4
    sim.set_timing(False)
    sim.step(2)
    assert all(n == 0 for ms, n in sim.read_timing().values())
    assert ddm.lib().ddm_set_timing(sim.ctx, 1 << 12) == ddm.DDM_EINVAL
