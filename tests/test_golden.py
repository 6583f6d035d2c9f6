"""Constants the paper prints, kept as cited text fixtures under tests/golden/,
against the optimiser, the treatment defaults, the library's configuration
defaults and the oracle's skill mapping.  CPU only."""
import inspect
import math
import pathlib

import numpy as np
import pytest

import workloads as W
from oracle import treatments as OT
from paper_2510_17335_amd import optim as O

GOLDEN = pathlib.Path(__file__).parent / "golden"


def _rows(name):
    out = []
    for line in (GOLDEN / name).read_text().splitlines():
        line = line.split("#", 1)[0].strip()
        if line:
            out.append(line.split())
    return out


def _table(name):
    return {r[0]: [float(v) for v in r[1:]] for r in _rows(name)}


def test_table1_steps_and_ranges():
    t = _table("table1_sysid.txt")
    assert set(t) == set(O.SYSID_STEPS) == set(O.SYSID_LO) == set(O.SYSID_HI)
    for k, (step, lo, hi) in t.items():
        assert O.SYSID_STEPS[k] == step, k
        assert O.SYSID_LO[k] == lo, k
        assert O.SYSID_HI[k] == hi, k


def test_optimiser_and_treatment_constants():
    t = _table("optimiser_constants.txt")
    spec = O.OptimSpec(free=["E"], step={"E": 1.0})
    assert spec.beta == t["rmsprop_beta"][0]
    assert list(O.LINE_SEARCH) == t["line_search_alphas"]
    assert list(spec.line_search) == t["line_search_alphas"]
    assert spec.clip == t["grad_clip"][0]
    # the default skill step is the printed 0.03 on the normalised parameters
    default = inspect.signature(O.skill_steps).parameters["theta_step"].default
    assert default == t["skill_step"][0]
    assert O.skill_steps() == O.skill_steps(t["skill_step"][0])
    # treatment thresholds: the oracle's and the binding's defaults
    assert (OT.CLIP, OT.OOM, OT.DELTA) == (t["grad_clip"][0], t["oom_star"][0], t["delta"][0])
    import paper_2510_17335_amd as m
    sig = inspect.signature(m.Simulator.set_grad_treatment).parameters
    assert (sig["clip"].default, sig["oom"].default, sig["delta"].default) == (OT.CLIP, OT.OOM, OT.DELTA)
    assert int(t["gradient_updates"][0]) == 20


@pytest.fixture(scope="module")
def orc():
    import oracle
    return oracle


@pytest.mark.parametrize("displace", [0.3, -0.4])
def test_demo_skill_against_appendix_a(orc, displace):
    """At the demonstration skill (with two displacements, which the paper
    derives from the target), the phase-1 actions carry the printed 0.12 per
    unit theta_displace, and phase 4 lifts by the printed d4."""
    t = _table("skill_demo.txt")
    theta = [displace, t["theta_rotate"][0], t["theta_insert_distance"][0], t["theta_push_distance"][0],
             t["theta_push_angle"][0]]
    d4 = t["lift_distance_m"][0]
    T, acts, jac = orc.skill_actions(theta, d4=d4)
    T1 = T[0]
    # x displacement of phase 1 (d1) and all entries of the phase-1 actions
    assert math.isclose(jac[:T1, 0, 0].sum(), t["dd1_dtheta_displace"][0], rel_tol=1e-12)
    assert math.isclose(jac[:T1, :, 0].sum(), t["dabar_dtheta_displace"][0], rel_tol=1e-12)
    assert np.all(jac[T1:, :, 0] == 0)
    # phase 4: the z actions (z up in the action frame) add up to the lift
    s4 = sum(T[:3])
    assert math.isclose(acts[s4:s4 + T[3], 2].sum(), d4, rel_tol=1e-12)


def test_lift_distance_defaults():
    d4 = _table("skill_demo.txt")["lift_distance_m"][0]
    import paper_2510_17335_amd as m
    assert inspect.signature(m.make_config).parameters["d_lift"].default == d4
    assert W.Workload.__dataclass_fields__["d_lift"].default == d4
    import oracle
    assert inspect.signature(oracle.skill_actions).parameters["d4"].default == d4
