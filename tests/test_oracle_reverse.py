"""Pins of the oracle's reverse-mode tape (the element-wise reference for the
gradient treatments of Sec. III-E):
  * untreated, its gradient equals the forward-mode (Dual<9>) gradient, which
    central differences pin, to 1e-10 on 2D and 3D tiny beds, with and
    without the shovel, from rest and from a strained state;
  * its treatment of one vector equals the Python statement of the three
    rules in oracle/treatments.py, whose own pins are worked examples;
  * its record of a treated vector's statistics is consistent with
    treated_stats of its record before the treatment;
  * thresholds that never act leave the gradient as it was.
CPU only."""
import numpy as np
import pytest

import workloads as W
from oracle import treatments as OT


def _case(orc, dim, shovel, pre, steps):
    w = W.tiny(dim, shovel=shovel, steps=pre + steps)
    w.precision = "f64"
    if w.target_seed is None:
        w.target_seed = 11
    x0, tg = W.bed_positions(w), W.target_heightmap(w)
    cfg = orc.config(w)
    s0 = orc.rollout(cfg, w.params, orc.initial_state(x0), pre)["state"] if pre else orc.initial_state(x0)
    return w, cfg, s0, tg


@pytest.mark.parametrize("dim,shovel,pre", [(2, False, 0), (2, False, 15), (3, False, 0), (3, True, 0), (3, True, 20)])
def test_reverse_tape_equals_forward_mode(orc, dim, shovel, pre):
    steps = 30
    w, cfg, s0, tg = _case(orc, dim, shovel, pre, steps)
    f = orc.rollout(cfg, w.params, s0, steps, step0=pre, target=tg, grad=True)
    r = orc.rollout_reverse(cfg, w.params, s0, steps, tg, step0=pre)
    assert r["loss"] == f["loss"]
    scale = np.abs(f["grad"]).max()
    assert scale > 0
    np.testing.assert_allclose(r["grad"], f["grad"], rtol=1e-10, atol=1e-10 * scale)
    if shovel:
        assert np.any(r["grad"][4:7] != 0)      # the blade turns in these sub-steps (skill phase 1)


@pytest.mark.parametrize("mode", ["clip", "scale", "norm"])
def test_vector_treatment_equals_python_rules(orc, mode):
    rng = np.random.default_rng(3)
    for mag in (1e-8, 1e-2, 1.0, 3.7e9, 1e14):
        g = rng.standard_normal(257) * mag
        for c, oom in ((1e4, 4.0), (0.5 * mag, 1.0), (2.0 * mag, -3.0)):
            want = OT.treat(g, mode, c=c, oom=oom, delta=1e-6)
            got = orc.treat(g, mode, clip=c, oom=oom, delta=1e-6)
            np.testing.assert_allclose(got, want, rtol=1e-15, atol=0.0)
    assert np.array_equal(orc.treat(np.zeros(5), "norm"), np.zeros(5))


@pytest.mark.parametrize("mode", ["clip", "scale", "norm"])
def test_treated_record_consistent(orc, mode):
    w, cfg, s0, tg = _case(orc, 3, True, 20, 20)
    r0 = orc.rollout_reverse(cfg, w.params, s0, 20, tg, step0=20, stats=True)
    amax = np.maximum(np.abs(r0["stats"][..., 0]), np.abs(r0["stats"][..., 1]))
    med = float(np.median(amax[amax > 0]))
    c, oom = 2.0 ** np.floor(np.log2(med)), float(np.round(np.log10(med)))
    r = orc.rollout_reverse(cfg, w.params, s0, 20, tg, step0=20, mode=mode, clip=c, oom=oom, stats=True)
    S = r["stats"]
    acted = 0
    for k in range(20):
        for v in range(6):
            pre, post = S[k, v, :3], S[k, v, 3:]
            want = OT.treated_stats(*pre, mode, c=c, oom=oom, delta=1e-6)
            for a in range(3):
                if want[a] is None:
                    assert post[a] <= pre[a] * (1 + 1e-12)
                else:
                    assert abs(post[a] - want[a]) <= 1e-13 * abs(want[a]), (k, v, a, post, want)
            acted += int(not np.array_equal(pre, post))
    assert acted > 0
    assert not np.allclose(r["grad"], r0["grad"], rtol=1e-6)


def test_idle_thresholds_keep_gradient(orc):
    w, cfg, s0, tg = _case(orc, 3, True, 20, 20)
    r0 = orc.rollout_reverse(cfg, w.params, s0, 20, tg, step0=20)
    for mode, kw in (("clip", {"clip": 1e300}), ("scale", {"oom": 300.0})):
        r = orc.rollout_reverse(cfg, w.params, s0, 20, tg, step0=20, mode=mode, **kw)
        assert np.array_equal(r["grad"], r0["grad"])
