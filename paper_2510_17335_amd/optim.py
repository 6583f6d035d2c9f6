"""Gradient-based system identification and skill optimisation on the batched
simulator (Sec. III-D, III-E, III-F; experiment design in Sec. IV-B).

- RMSprop with beta = 0.9 on the free parameters; per-parameter step sizes in
  parameter units (Table I for E, nu, rho, phi_f; the skill step of 0.03 on the
  normalised skill parameters of Eqs. d1-d3, converted to physical units by
  `skill_steps`).
- The gradient treatments of Sec. III-E inside the reverse pass (clipping of
  the particle and grid adjoints at 1e4 is the paper's best setting), passed
  to `GpuEvaluator` as `treatment`; and, on top, an element-wise clip of the
  parameter gradients at `OptimSpec.clip` (1e4 by default, inf disables it).
- A line search before each update (Sec. III-F): the update is scaled by
  alpha in {0.1, 0.5, 1.0, 1.5, 2.0}; the five candidates are run as five
  instances of one batched forward launch and the one with the lowest loss is
  taken.
- Loss-landscape sweeps as batched forwards over a list of parameter sets.

Parameters are the 9-vectors [E, nu, phi_deg, rho, depth, angle_deg, push,
displace, push_angle_deg] of the library's gradient.  The driver itself only needs two evaluators:
loss and gradient at one parameter set, and the losses of a batch of
parameter sets; `GpuEvaluator` provides both on the GPU.
"""
from __future__ import annotations

import copy
import math
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

PARAM_NAMES = ("E", "nu", "phi_deg", "rho", "depth", "angle_deg", "push", "displace", "push_angle_deg")
LINE_SEARCH = (0.1, 0.5, 1.0, 1.5, 2.0)

# Table I: step sizes and ranges of the physics parameters.  The table gives
# E in kPa with values of 5e4-2e5; the workloads here are in Pa with E of
# 1e4-1e6, so the numbers are read as Pa.
SYSID_STEPS = {"E": 1e4, "nu": 0.01, "rho": 50.0, "phi_deg": 1.0}
SYSID_LO = {"E": 5e4, "nu": 0.1, "rho": 1200.0, "phi_deg": 10.0}
SYSID_HI = {"E": 2e5, "nu": 0.4, "rho": 2200.0, "phi_deg": 40.0}


def skill_steps(theta_step: float = 0.03) -> Dict[str, float]:
    """The step on the normalised skill parameters (Sec. IV-C: 0.03) in
    physical units: d1 = 0.12 theta m, phi1 = theta pi/3 rad = 60 theta deg,
    d2 = 0.03 (theta + 1) m, d3 = 0.1 (theta + 1) + 0.04 m, phi3 = (theta + 3)
    pi/3 rad = 60 (theta + 3) deg (Eqs. d1-d3)."""
    return {"depth": 0.03 * theta_step, "angle_deg": 60.0 * theta_step, "push": 0.1 * theta_step,
            "displace": 0.12 * theta_step, "push_angle_deg": 60.0 * theta_step}


@dataclass
class OptimSpec:
    free: Sequence[str]
    step: Dict[str, float]
    lo: Dict[str, float] = field(default_factory=dict)
    hi: Dict[str, float] = field(default_factory=dict)
    beta: float = 0.9
    eps: float = 1e-8
    clip: float = 1e4
    line_search: Sequence[float] = LINE_SEARCH

    def index(self) -> List[int]:
        return [PARAM_NAMES.index(n) for n in self.free]


@dataclass
class OptimState:
    theta: np.ndarray                 # full parameter vector (PARAM_NAMES)
    v: np.ndarray                     # RMSprop second moment of the free parameters
    history: List[dict] = field(default_factory=list)


def clamp(theta: np.ndarray, spec: OptimSpec) -> np.ndarray:
    out = theta.copy()
    for k, n in zip(spec.index(), spec.free):
        if n in spec.lo:
            out[k] = max(out[k], spec.lo[n])
        if n in spec.hi:
            out[k] = min(out[k], spec.hi[n])
    return out


def rmsprop_direction(g: np.ndarray, v: np.ndarray, spec: OptimSpec) -> Tuple[np.ndarray, np.ndarray]:
    """Clipped gradient -> (new second moment, update direction) of the free
    parameters; the update is theta - alpha * direction."""
    g = np.clip(g, -spec.clip, spec.clip)
    v = spec.beta * v + (1.0 - spec.beta) * g * g
    step = np.array([spec.step[n] for n in spec.free])
    return v, step * g / (np.sqrt(v) + spec.eps)


def optimise(theta0: Sequence[float], spec: OptimSpec, grad_fn: Callable[[np.ndarray], Tuple[float, np.ndarray]],
             batch_loss_fn: Callable[[List[np.ndarray]], np.ndarray], iterations: int,
             callback: Optional[Callable[[dict], None]] = None) -> OptimState:
    """RMSprop with line search.  grad_fn(theta) -> (loss, grad[len(PARAM_NAMES)]);
    batch_loss_fn([theta, ...]) -> losses (one batched forward)."""
    idx = spec.index()
    st = OptimState(theta=clamp(np.asarray(theta0, dtype=np.float64), spec), v=np.zeros(len(idx)))
    for it in range(iterations):
        loss, grad = grad_fn(st.theta)
        g = np.asarray(grad, dtype=np.float64)[idx]
        st.v, d = rmsprop_direction(g, st.v, spec)
        cands = []
        for a in spec.line_search:
            th = st.theta.copy()
            th[idx] = th[idx] - a * d
            cands.append(clamp(th, spec))
        losses = np.asarray(batch_loss_fn(cands), dtype=np.float64)
        best = int(np.argmin(losses))
        rec = {"iteration": it, "loss": float(loss), "grad": np.asarray(grad, dtype=np.float64).copy(),
               "alphas": list(spec.line_search), "candidate_losses": losses.copy(), "chosen": best,
               "theta": cands[best].copy()}
        st.history.append(rec)
        st.theta = cands[best]
        if callback:
            callback(rec)
    return st


# ---------------------------------------------------------------------------
# GPU evaluators
# ---------------------------------------------------------------------------

def instance_with(ddm, base, theta: Sequence[float]):
    """A copy of a ddm_instance with the parameters (PARAM_NAMES order) replaced."""
    inst = copy.copy(base)
    inst.E, inst.nu, inst.phi_deg, inst.rho = float(theta[0]), float(theta[1]), float(theta[2]), float(theta[3])
    inst.depth, inst.angle_deg, inst.push = float(theta[4]), float(theta[5]), float(theta[6])
    if len(theta) > 7:
        inst.displace, inst.push_angle_deg = float(theta[7]), float(theta[8])
    return inst


class GpuEvaluator:
    """Loss/gradient at one parameter set (a recorded rollout and the reverse
    pass on a one-instance context) and batched losses (forward only, on a
    context of `batch` instances of the same bed), for one workload, its
    initial positions x0 and a target height map."""

    def __init__(self, ddm, w, x0: np.ndarray, target: np.ndarray, steps: int, batch: int = len(LINE_SEARCH),
                 checkpoint_every: int = 50, precision: Optional[str] = None, sort_every: int = 8,
                 treatment: Optional[dict] = None):
        """treatment: keyword arguments of Simulator.set_grad_treatment for
        the gradient passes, e.g. {"mode": "clip", "clip": 1e4}."""
        self.ddm = ddm
        self.steps = steps
        cfg, inst = ddm.from_workload(w, max_steps=steps, checkpoint_every=checkpoint_every, precision=precision,
                                      sort_every=sort_every)
        self.base = inst
        self.grad_sim = ddm.Simulator(cfg, [inst])
        if treatment:
            self.grad_sim.set_grad_treatment(**treatment)
        self.batch = batch
        self.batch_sim = ddm.Simulator(cfg, [inst] * batch)
        # the inputs stay in device memory, in the contexts' precision
        torch, dev, dt = self.grad_sim.torch, self.grad_sim.device, self.grad_sim.dtype
        x0 = np.asarray(x0)
        self.x0 = torch.as_tensor(x0, device=dev).to(dt)
        self.x0_batch = torch.as_tensor(np.concatenate([x0] * batch), device=dev).to(dt)
        target = np.asarray(target, dtype=np.float64).reshape(1, -1)
        self.target = torch.as_tensor(target, device=dev)
        self.target_batch = torch.as_tensor(np.repeat(target, batch, axis=0), device=dev)
        self.passes = 0

    def grad(self, theta: np.ndarray) -> Tuple[float, np.ndarray]:
        sim = self.grad_sim
        sim.set_instances([instance_with(self.ddm, self.base, theta)])
        sim.init_state(self.x0)
        sim.rollout(self.steps)
        loss = float(sim.loss(self.target)[0])
        g = sim.backward()[0].cpu().numpy()
        self.passes += 1
        return loss, g

    def losses(self, thetas: List[np.ndarray]) -> np.ndarray:
        out = []
        for i in range(0, len(thetas), self.batch):
            chunk = list(thetas[i:i + self.batch])
            n = len(chunk)
            chunk += [chunk[-1]] * (self.batch - n)          # pad the last launch
            sim = self.batch_sim
            sim.set_instances([instance_with(self.ddm, self.base, th) for th in chunk])
            sim.init_state(self.x0_batch)
            sim.step(self.steps)
            out.append(sim.loss(self.target_batch).cpu().numpy()[:n])
            self.passes += 1
        return np.concatenate(out)


def landscape(evaluator: GpuEvaluator, thetas: List[np.ndarray]) -> np.ndarray:
    """Losses over a list of parameter sets, `evaluator.batch` per forward launch."""
    return evaluator.losses(list(thetas))
