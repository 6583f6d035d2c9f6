"""Python binding of libddmpm.so (differentiable MLS-MPM sand digging on MI355X).

Argument marshalling only: every step of the simulation, the loss and the
reverse pass runs in the library's HIP kernels.  PyTorch provides device
memory (the workspace is one uint8 tensor) and the stream.  If the library is
not built, importing works but creating a Simulator raises.

The calls mirror include/ddmpm.h: validate_config, workspace_query, create,
init_state, step, rollout, loss, backward, get_state / set_state, get_grid,
get_heightmap, check.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libddmpm.so")

DDM_OK, DDM_EINVAL, DDM_ENOMEM, DDM_EDEVICE, DDM_ENAN, DDM_EDOMAIN, DDM_ESTATE = range(7)
DDM_F32, DDM_F64 = 0, 1
TIMING_ALL = 0x3FF          # DDM_TIMING_ALL: every launch group
# Differentiable inputs, in the order of every gradient (DDM_N_PARAMS).
PARAM_NAMES = ("E", "nu", "phi_deg", "rho", "depth", "angle_deg", "push", "displace", "push_angle_deg")
N_PARAMS = len(PARAM_NAMES)


class DdmConfig(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("n_grid", C.c_int32), ("bound", C.c_int32), ("precision", C.c_int32),
        ("n_sub", C.c_int32), ("shovel", C.c_int32), ("hm_res", C.c_int32), ("region_sign", C.c_int32),
        ("gravity", C.c_double), ("ppc", C.c_double), ("shovel_half", C.c_double * 3),
        ("contact_skin", C.c_double), ("shovel_mu", C.c_double), ("v_lin", C.c_double),
        ("v_ang", C.c_double), ("d_lift", C.c_double), ("hm_origin", C.c_double * 2), ("hm_size", C.c_double),
        ("hm_offset", C.c_double), ("region_depth", C.c_double), ("m_target", C.c_double), ("m_ref", C.c_double),
        ("w_mass", C.c_double), ("w_hm", C.c_double), ("checkpoint_every", C.c_int32), ("max_steps", C.c_int32),
        ("sort_every", C.c_int32), ("skill_unrounded", C.c_int32), ("particle_contact", C.c_int32),
        ("record_segments", C.c_int32), ("w_emd", C.c_double), ("tile_workgroups", C.c_int32), ("grid_record_blocks", C.c_int32),
        ("deterministic", C.c_int32),
    ]


class DdmInstance(C.Structure):
    _fields_ = [
        ("n_particles", C.c_int64), ("E", C.c_double), ("nu", C.c_double), ("phi_deg", C.c_double),
        ("rho", C.c_double), ("cohesion", C.c_double), ("depth", C.c_double), ("angle_deg", C.c_double),
        ("push", C.c_double), ("dt", C.c_double), ("tip0", C.c_double * 3), ("displace", C.c_double),
        ("push_angle_deg", C.c_double),
    ]


class DdmSizes(C.Structure):
    _fields_ = [("workspace_bytes", C.c_size_t), ("state_bytes", C.c_size_t), ("padded_particles", C.c_int64)]


class DdmDeviceError(C.Structure):
    _fields_ = [("flags", C.c_uint32), ("first_instance", C.c_uint32), ("clamp_count", C.c_uint64)]


# Gradient treatments of the reverse pass and the adjoint vectors they act on
# (ddm_set_grad_treatment).
TREATMENTS = ("none", "clip", "scale", "norm")
TREAT_VARS = ("x", "v", "F", "grid_v_post", "grid_mv", "grid_m")


class DdmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ddmpm error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded library; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() (hipcc, gfx950) first")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        cfgp, instp = C.POINTER(DdmConfig), C.POINTER(DdmInstance)
        sig = {
            "ddm_validate_config": (C.c_int, [cfgp, i32, instp, C.c_char_p, C.c_size_t]),
            "ddm_workspace_query": (C.c_int, [cfgp, i32, instp, C.POINTER(DdmSizes)]),
            "ddm_skill_pose_table": (C.c_int, [cfgp, instp, i32, vp, vp]),
            "ddm_create": (C.c_int, [cfgp, i32, instp, vp, C.c_size_t, vp, C.POINTER(vp)]),
            "ddm_init_state": (C.c_int, [vp, vp]),
            "ddm_set_instances": (C.c_int, [vp, i32, instp]),
            "ddm_step": (C.c_int, [vp, i32]),
            "ddm_rollout": (C.c_int, [vp, i32]),
            "ddm_loss": (C.c_int, [vp, vp, vp]),
            "ddm_set_emd_target": (C.c_int, [vp, vp, i32]),
            "ddm_backward": (C.c_int, [vp, vp, vp]),
            "ddm_pass": (C.c_int, [vp, vp, i32, vp, vp, vp, vp, i32]),
            "ddm_autotune": (C.c_int, [vp, C.c_char_p, C.POINTER(i32)]),
            "ddm_get_launch": (C.c_int, [vp, C.POINTER(i32), C.POINTER(i32)]),
            "ddm_get_state": (C.c_int, [vp, vp]),
            "ddm_set_state": (C.c_int, [vp, vp]),
            "ddm_get_grid": (C.c_int, [vp, vp]),
            "ddm_bin_keys": (C.c_int, [vp, vp, vp]),
            "ddm_get_heightmap": (C.c_int, [vp, vp]),
            "ddm_eval_math": (C.c_int, [i32, vp, vp, i64, vp]),
            "ddm_loss_noalloc": (C.c_int, [cfgp, instp, i32, vp, vp, vp, vp, vp]),
            "ddm_check": (C.c_int, [vp, C.POINTER(DdmDeviceError)]),
            "ddm_diagnostics": (C.c_int, [vp, vp]),
            "ddm_steps_taken": (i64, [vp]),
            "ddm_instance_offset": (i64, [vp, i32]),
            "ddm_set_grad_treatment": (C.c_int, [vp, i32, C.c_double, C.c_double, C.c_double, vp, i32]),
            "ddm_set_timing": (C.c_int, [vp, i32]),
            "ddm_read_timing": (C.c_int, [vp, i32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
            "ddm_destroy": (None, [vp]),
            "ddm_status_str": (C.c_char_p, [C.c_int]),
            "ddm_last_error": (C.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int):
    if rc != DDM_OK:
        L = lib()
        raise DdmError(rc, f"{L.ddm_status_str(rc).decode()}: {L.ddm_last_error().decode()}")


# ---------------------------------------------------------------------------
# Configuration helpers
# ---------------------------------------------------------------------------

def make_config(dim: int, n_grid: int, precision: str = "f32", *, bound: int = 3, n_sub: int = 10,
                shovel: bool = False, gravity: float = -9.8, ppc: float = 8.0,
                shovel_half=(0.05, 0.0025, 0.04), contact_skin: Optional[float] = None, shovel_mu: float = 0.5,
                v_lin: float = 3.0, v_ang: float = 10 * math.pi, d_lift: float = 0.01, hm_res: int = 40,
                hm_origin=(0.2, 0.2), hm_size: float = 0.6, hm_offset: Optional[float] = None,
                region_depth: float = 0.03, m_target: float = 0.192, m_ref: float = 0.384, w_mass: float = 1.0,
                w_hm: float = 1.0, region_sign: int = -1, checkpoint_every: int = 50,
                max_steps: int = 1000, sort_every: int = 8, skill_unrounded: bool = False,
                particle_contact: bool = False, w_emd: float = 0.0, record_segments: int = 1,
                deterministic: bool = False) -> DdmConfig:
    c = DdmConfig()
    c.dim, c.n_grid, c.bound = dim, n_grid, bound
    c.precision = DDM_F64 if precision == "f64" else DDM_F32
    c.n_sub, c.shovel, c.hm_res, c.region_sign = n_sub, int(shovel), hm_res, region_sign
    c.gravity, c.ppc = gravity, float(ppc)
    for k in range(3):
        c.shovel_half[k] = shovel_half[k]
    c.contact_skin = 1.0 / n_grid if contact_skin is None else contact_skin
    c.shovel_mu, c.v_lin, c.v_ang, c.d_lift = shovel_mu, v_lin, v_ang, d_lift
    c.hm_origin[0], c.hm_origin[1] = hm_origin
    c.hm_size = hm_size
    c.hm_offset = (1.0 / n_grid) / round(ppc ** (1.0 / dim)) if hm_offset is None else hm_offset
    c.region_depth, c.m_target, c.m_ref, c.w_mass, c.w_hm = region_depth, m_target, m_ref, w_mass, w_hm
    c.checkpoint_every, c.max_steps, c.sort_every = checkpoint_every, max_steps, sort_every
    c.skill_unrounded, c.particle_contact = int(bool(skill_unrounded)), int(bool(particle_contact))
    c.w_emd = float(w_emd)
    c.record_segments = int(record_segments)
    c.deterministic = int(bool(deterministic))
    return c


def make_instance(n_particles: int, *, E=3.5e5, nu=0.3, phi_deg=30.0, rho=1600.0, cohesion=0.0, depth=0.05,
                  angle_deg=30.0, push=0.15, dt=2e-4, tip0=(0.5, 0.34375, 0.5), displace=0.0,
                  push_angle_deg=180.0) -> DdmInstance:
    s = DdmInstance()
    s.n_particles = int(n_particles)
    s.E, s.nu, s.phi_deg, s.rho, s.cohesion = E, nu, phi_deg, rho, cohesion
    s.depth, s.angle_deg, s.push, s.dt = depth, angle_deg, push, dt
    s.displace, s.push_angle_deg = displace, push_angle_deg
    t = list(tip0) + [0.0] * (3 - len(tip0))
    for k in range(3):
        s.tip0[k] = t[k]
    return s


def from_workload(w, max_steps: Optional[int] = None, checkpoint_every: Optional[int] = None,
                  precision: Optional[str] = None, sort_every: int = 8, deterministic: bool = False):
    """(config, instance) for an object with the attributes of a workload
    description (dim, n_grid, dt, ppc, material, skill, ...)."""
    cfg = make_config(
        w.dim, w.n_grid, precision or w.precision, bound=w.bound, n_sub=w.n_sub, shovel=w.skill is not None,
        gravity=w.gravity, ppc=w.ppc, shovel_half=w.shovel_half, contact_skin=w.skin, shovel_mu=w.mu_b,
        v_lin=w.v_l, v_ang=w.v_w, d_lift=w.d_lift, hm_res=w.hm_res, hm_origin=w.hm_origin, hm_size=w.hm_size,
        hm_offset=w.hm_offset, region_depth=w.region_depth, m_target=w.m_target, m_ref=w.m_ref, w_mass=w.w_mass,
        w_hm=w.w_hm, region_sign=w.region_sign,
        checkpoint_every=checkpoint_every or w.checkpoint_every or 50,
        max_steps=max_steps or w.steps, sort_every=sort_every, skill_unrounded=w.skill_unrounded,
        particle_contact=w.particle_contact, w_emd=w.w_emd, deterministic=deterministic)
    p = w.params
    inst = make_instance(w.n_particles, E=p[0], nu=p[1], phi_deg=p[2], rho=p[3], cohesion=w.material.cohesion,
                         depth=p[4], angle_deg=p[5], push=p[6], dt=w.dt, tip0=w.tip0, displace=p[7],
                         push_angle_deg=p[8])
    return cfg, inst


MATH_FUNCTIONS = ("log1p", "expm1")


def eval_math(fn: str, x):
    """The FP32 log1p or expm1 of the device kernels applied to a float32
    CUDA tensor (ddm_eval_math), on the current stream; returns a new tensor."""
    import torch
    if x.dtype != torch.float32 or not x.is_cuda:
        raise ValueError("x must be a float32 CUDA tensor")
    x = x.contiguous()
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream(x.device)
    _check(lib().ddm_eval_math(MATH_FUNCTIONS.index(fn), C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                               x.numel(), C.c_void_p(stream.cuda_stream)))
    return y


def loss_noalloc(cfg: DdmConfig, inst: DdmInstance, final_step: int, x, target, hm=True):
    """ddm_loss_noalloc on the current stream: the loss (and height map) of one
    instance's positions x [n, dim] (CUDA tensor of the context precision)
    with the blade after sub-step final_step (-1: the initial pose), without a
    context or any allocation inside the library.  Returns (loss [1], hm or None)."""
    import torch
    dt = torch.float64 if cfg.precision == DDM_F64 else torch.float32
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == dt):
        raise ValueError("x must be a CUDA tensor of the configuration's precision")
    x = x.contiguous()
    tg = torch.as_tensor(target, dtype=torch.float64).to(x.device).contiguous()
    loss = torch.empty(1, dtype=torch.float64, device=x.device)
    out = torch.empty(tg.numel(), dtype=torch.float64, device=x.device) if hm else None
    stream = torch.cuda.current_stream(x.device)
    _check(lib().ddm_loss_noalloc(C.byref(cfg), C.byref(inst), int(final_step), C.c_void_p(x.data_ptr()),
                                  C.c_void_p(tg.data_ptr()), C.c_void_p(loss.data_ptr()),
                                  C.c_void_p(out.data_ptr()) if hm else None, C.c_void_p(stream.cuda_stream)))
    return loss, out


def skill_pose_table(cfg: DdmConfig, inst: DdmInstance, n_steps: int):
    """(pose [n_steps, 8], jacobian [n_steps, 8, 5]) of one instance's skill,
    computed on the host by the library (ddm_skill_pose_table)."""
    pose = np.zeros((n_steps, 8))
    jac = np.zeros((n_steps, 8, 5))
    _check(lib().ddm_skill_pose_table(C.byref(cfg), C.byref(inst), int(n_steps), C.c_void_p(pose.ctypes.data),
                                      C.c_void_p(jac.ctypes.data)))
    return pose, jac


def validate_config(cfg: DdmConfig, instances: Sequence[DdmInstance]) -> str:
    """Empty string when valid, else the library's message (host only)."""
    arr = (DdmInstance * len(instances))(*instances)
    buf = C.create_string_buffer(512)
    rc = lib().ddm_validate_config(C.byref(cfg), len(instances), arr, buf, 512)
    return "" if rc == DDM_OK else buf.value.decode()


def workspace_query(cfg: DdmConfig, instances: Sequence[DdmInstance]) -> DdmSizes:
    arr = (DdmInstance * len(instances))(*instances)
    out = DdmSizes()
    _check(lib().ddm_workspace_query(C.byref(cfg), len(instances), arr, C.byref(out)))
    return out


# ---------------------------------------------------------------------------
# Simulator
# ---------------------------------------------------------------------------

class Simulator:
    """One library context: n instances sharing a configuration."""

    def __init__(self, cfg: DdmConfig, instances: Sequence[DdmInstance], device="cuda", stream=None):
        import torch
        self.torch = torch
        self.cfg = cfg
        self.instances = list(instances)
        self.n_inst = len(self.instances)
        self.device = torch.device(device)
        self.dtype = torch.float64 if cfg.precision == DDM_F64 else torch.float32
        self.dim = cfg.dim
        self.sizes = workspace_query(cfg, self.instances)
        self.workspace = torch.empty(int(self.sizes.workspace_bytes), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        arr = (DdmInstance * self.n_inst)(*self.instances)
        ctx = C.c_void_p()
        _check(lib().ddm_create(C.byref(cfg), self.n_inst, arr, C.c_void_p(self.workspace.data_ptr()),
                                int(self.sizes.workspace_bytes), C.c_void_p(self.stream.cuda_stream), C.byref(ctx)))
        self.ctx = ctx
        self.offsets = [int(lib().ddm_instance_offset(ctx, i)) for i in range(self.n_inst)]
        self.counts = [int(s.n_particles) for s in self.instances]
        self.npix = cfg.hm_res ** (cfg.dim - 1)

    # Stream order between torch's current stream (where tensors given to and
    # returned by these methods are produced and consumed) and the context's
    # stream, when they differ.
    def _inputs_ready(self):
        cur = self.torch.cuda.current_stream(self.device)
        if cur != self.stream:
            self.stream.wait_stream(cur)

    def _outputs_ready(self):
        cur = self.torch.cuda.current_stream(self.device)
        if cur != self.stream:
            cur.wait_stream(self.stream)

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx and _lib is not None:
            try:
                self.stream.synchronize()
                _lib.ddm_destroy(ctx)
            except Exception:
                pass
            self.ctx = None

    def set_instances(self, instances: Sequence[DdmInstance]):
        """New per-instance parameters (same count and particle counts), e.g.
        the candidates of an optimiser step (ddm_set_instances)."""
        instances = list(instances)
        arr = (DdmInstance * len(instances))(*instances)
        _check(lib().ddm_set_instances(self.ctx, len(instances), arr))
        self.instances = instances

    # -- state ---------------------------------------------------------------
    @property
    def state_rows(self) -> int:
        d = self.dim
        return 2 * d + 2 * d * d

    def init_state(self, x0):
        """x0: [sum N_i, dim] positions (numpy or torch), instances concatenated."""
        t = self.torch
        x0 = t.as_tensor(np.asarray(x0) if not isinstance(x0, t.Tensor) else x0)
        self._x0 = x0.to(device=self.device, dtype=self.dtype).contiguous()
        assert self._x0.shape == (sum(self.counts), self.dim)
        self._inputs_ready()
        _check(lib().ddm_init_state(self.ctx, C.c_void_p(self._x0.data_ptr())))

    def step(self, n: int):
        _check(lib().ddm_step(self.ctx, int(n)))

    def rollout(self, n: int):
        _check(lib().ddm_rollout(self.ctx, int(n)))

    @property
    def steps_taken(self) -> int:
        return int(lib().ddm_steps_taken(self.ctx))

    def get_state(self):
        """Raw [rows, padded_particles] state tensor (a copy)."""
        out = self.torch.empty((self.state_rows, int(self.sizes.padded_particles)), dtype=self.dtype,
                               device=self.device)
        self._inputs_ready()
        _check(lib().ddm_get_state(self.ctx, C.c_void_p(out.data_ptr())))
        self._outputs_ready()
        return out

    def set_state(self, state):
        state = state.to(device=self.device, dtype=self.dtype).contiguous()
        assert state.shape == (self.state_rows, int(self.sizes.padded_particles))
        self._set_state_keep = state
        self._inputs_ready()
        _check(lib().ddm_set_state(self.ctx, C.c_void_p(state.data_ptr())))

    def instance_state(self, state, i: int):
        """(x, v, C, F) of instance i as float64 [N, dim], [N, dim], [N, dim, dim],
        [N, dim, dim], decoded from a raw state: in FP32 the position rows hold
        32-bit fixed point (x = value * 2^-32), and the last rows hold F - I."""
        t = self.torch
        d, o, n = self.dim, self.offsets[i], self.counts[i]
        s = state[:, o:o + n]
        if self.dtype == t.float32:
            xi = s[:d].contiguous().view(t.int32).to(t.int64) & 0xFFFFFFFF
            x = (xi.double() * 2.0 ** -32).T
        else:
            x = s[:d].double().T
        v = s[d:2 * d].double().T
        Cm = s[2 * d:2 * d + d * d].double().T.reshape(n, d, d)
        F = s[2 * d + d * d:].double().T.reshape(n, d, d) + t.eye(d, dtype=t.float64, device=s.device)
        return x, v, Cm, F

    def packed_state(self, i: int = 0) -> np.ndarray:
        """Instance i as a float64 [N, 2d + 2d^2] array (x, v, C, F per particle)."""
        st = self.get_state()
        x, v, Cm, F = self.instance_state(st, i)
        n = self.counts[i]
        out = self.torch.cat([x, v, Cm.reshape(n, -1), F.reshape(n, -1)], dim=1)
        return out.cpu().numpy()

    def bin_keys(self):
        """(keys, perm) of the current state's slots, uint32 numpy arrays."""
        t = self.torch
        n = int(self.sizes.padded_particles)
        keys = t.empty(n, dtype=t.int32, device=self.device)
        perm = t.empty(n, dtype=t.int32, device=self.device)
        self._inputs_ready()
        _check(lib().ddm_bin_keys(self.ctx, C.c_void_p(keys.data_ptr()), C.c_void_p(perm.data_ptr())))
        self._outputs_ready()
        return keys.cpu().numpy().view(np.uint32), perm.cpu().numpy().view(np.uint32)

    def get_grid(self):
        nodes = self.cfg.n_grid ** self.dim
        out = self.torch.empty((self.n_inst, nodes, 8), dtype=self.dtype, device=self.device)
        self._inputs_ready()
        _check(lib().ddm_get_grid(self.ctx, C.c_void_p(out.data_ptr())))
        self._outputs_ready()
        return out

    # -- loss and gradient ---------------------------------------------------
    def loss(self, target):
        """target: [n_inst, npix] float64 (numpy or torch). Returns loss [n_inst] (device, float64)."""
        t = self.torch
        tg = t.as_tensor(np.asarray(target) if not isinstance(target, t.Tensor) else target)
        self._target = tg.to(device=self.device, dtype=t.float64).reshape(self.n_inst, self.npix).contiguous()
        out = t.empty(self.n_inst, dtype=t.float64, device=self.device)
        self._inputs_ready()
        _check(lib().ddm_loss(self.ctx, C.c_void_p(self._target.data_ptr()), C.c_void_p(out.data_ptr())))
        self._outputs_ready()
        return out

    def set_emd_target(self, points):
        """Target point clouds of the EMD term, [n_inst, m, 3] or [m, 3] for
        every instance (ddm_set_emd_target)."""
        t = self.torch
        pts = t.as_tensor(np.asarray(points) if not isinstance(points, t.Tensor) else points, dtype=t.float64)
        if pts.dim() == 2:
            pts = pts.unsqueeze(0).expand(self.n_inst, -1, -1)
        self._emd_target = pts.to(self.device).contiguous()
        self._inputs_ready()
        _check(lib().ddm_set_emd_target(self.ctx, C.c_void_p(self._emd_target.data_ptr()), int(pts.shape[1])))

    def heightmap(self):
        out = self.torch.empty((self.n_inst, self.npix), dtype=self.torch.float64, device=self.device)
        self._inputs_ready()
        _check(lib().ddm_get_heightmap(self.ctx, C.c_void_p(out.data_ptr())))
        self._outputs_ready()
        return out

    def backward(self, dloss=None):
        """Gradient [n_inst, N_PARAMS] of sum(dloss * loss) w.r.t. PARAM_NAMES."""
        t = self.torch
        if dloss is None:
            dloss = t.ones(self.n_inst, dtype=t.float64, device=self.device)
        dl = t.as_tensor(dloss, dtype=t.float64).to(self.device).contiguous()
        grad = t.empty((self.n_inst, N_PARAMS), dtype=t.float64, device=self.device)
        self._inputs_ready()
        _check(lib().ddm_backward(self.ctx, C.c_void_p(dl.data_ptr()), C.c_void_p(grad.data_ptr())))
        self._keep = dl
        self._outputs_ready()
        return grad

    def full_pass(self, x0, n: int, target, dloss=None, graph: bool = False):
        """init_state(x0) + rollout(n) + loss(target) + backward(dloss) as one
        library call (ddm_pass).  graph=True captures the pass into a HIP graph
        on the first call and replays it on later calls; the inputs are copied
        into buffers this Simulator keeps, so the graph sees fixed pointers.
        Needs a Simulator created on a non-default stream for graph=True.
        Returns (loss [n_inst], grad [n_inst, N_PARAMS]), device tensors that the next
        pass overwrites."""
        t = self.torch
        if not hasattr(self, "_pass_bufs"):
            self._pass_bufs = {
                "x0": t.empty((sum(self.counts), self.dim), dtype=self.dtype, device=self.device),
                "tg": t.empty((self.n_inst, self.npix), dtype=t.float64, device=self.device),
                "dl": t.empty(self.n_inst, dtype=t.float64, device=self.device),
                "loss": t.empty(self.n_inst, dtype=t.float64, device=self.device),
                "grad": t.empty((self.n_inst, N_PARAMS), dtype=t.float64, device=self.device),
            }
        B = self._pass_bufs
        self._inputs_ready()
        with t.cuda.stream(self.stream):
            B["x0"].copy_(t.as_tensor(np.asarray(x0) if not isinstance(x0, t.Tensor) else x0).reshape(B["x0"].shape))
            B["tg"].copy_(t.as_tensor(np.asarray(target) if not isinstance(target, t.Tensor) else target)
                          .reshape(B["tg"].shape))
            if dloss is None:
                B["dl"].fill_(1.0)
            else:
                B["dl"].copy_(t.as_tensor(dloss, dtype=t.float64))
        ptr = {k: C.c_void_p(v.data_ptr()) for k, v in B.items()}
        _check(lib().ddm_pass(self.ctx, ptr["x0"], int(n), ptr["tg"], ptr["dl"], ptr["loss"], ptr["grad"],
                              int(bool(graph))))
        self._outputs_ready()
        return B["loss"], B["grad"]

    def autotune(self, cache_path: Optional[str] = None) -> int:
        """Chooses and sets the binning interval and the tile kernels'
        workgroup count (ddm_autotune); returns the interval (see launch())."""
        r = C.c_int32()
        _check(lib().ddm_autotune(self.ctx, cache_path.encode() if cache_path else None, C.byref(r)))
        return int(r.value)

    def launch(self):
        """(binning interval, tile-kernel workgroups; 0 = about one per tile) of the context."""
        r, w = C.c_int32(), C.c_int32()
        _check(lib().ddm_get_launch(self.ctx, C.byref(r), C.byref(w)))
        return int(r.value), int(w.value)

    TIMING_GROUPS = ("p2g", "grid_update", "g2p", "binning", "g2p_adj", "grid_adj", "p2g_adj", "clear", "loss",
                     "treat")

    # -- gradient treatments (Sec. III-E) --------------------------------------
    def set_grad_treatment(self, mode: str = "none", clip: float = 1e4, oom: float = 4.0, delta: float = 1e-6,
                           record_steps: int = 0):
        """Treatment of the adjoint vectors inside every later backward pass
        (ddm_set_grad_treatment): mode in TREATMENTS; record_steps > 0 keeps
        the max / min / 2-norm of each vector before and after its treatment
        for sub-steps 0 .. record_steps-1, read back with grad_stats()."""
        t = self.torch
        code = TREATMENTS.index(mode)
        self._stats = (t.zeros((record_steps, self.n_inst, len(TREAT_VARS), 6), dtype=t.float64, device=self.device)
                       if record_steps > 0 else None)
        ptr = C.c_void_p(self._stats.data_ptr()) if self._stats is not None else None
        self._inputs_ready()
        _check(lib().ddm_set_grad_treatment(self.ctx, code, float(clip), float(oom), float(delta), ptr,
                                            int(record_steps)))

    def grad_stats(self) -> np.ndarray:
        """[record_steps, n_inst, 6 variables (TREAT_VARS), 6] of the last
        backward pass: max, min, 2-norm before the treatment, then after it."""
        if getattr(self, "_stats", None) is None:
            raise RuntimeError("no statistics recorded: set_grad_treatment(record_steps=...) first")
        self._outputs_ready()
        return self._stats.cpu().numpy()

    def grad_growth(self, segment: Optional[int] = None) -> np.ndarray:
        """Growth of the adjoints backwards in time, per segment of `segment`
        sub-steps (the checkpoint interval by default): [n_segments, n_inst,
        6 variables, 2] = the largest magnitude and the largest 2-norm of each
        variable's adjoint over the segment's sub-steps, before treatment."""
        S = self.grad_stats()
        seg = int(segment or self.cfg.checkpoint_every)
        amax = np.maximum(np.abs(S[..., 0]), np.abs(S[..., 1]))
        out = []
        for k in range(0, S.shape[0], seg):
            out.append(np.stack([amax[k:k + seg].max(axis=0), S[k:k + seg, ..., 2].max(axis=0)], axis=-1))
        return np.stack(out)

    def set_timing(self, enable=True, groups=None):
        """Time launch groups with HIP events: every group (enable=True), none
        (False), or the named groups of TIMING_GROUPS (groups=[...]).  Each
        event pair costs a few microseconds of stream time."""
        if groups is not None:
            mask = 0
            for g in groups:
                mask |= 1 << self.TIMING_GROUPS.index(g)
        else:
            mask = TIMING_ALL if enable else 0
        _check(lib().ddm_set_timing(self.ctx, mask))

    def read_timing(self) -> dict:
        """{group: (total_ms, launches)} since timing was enabled."""
        out = {}
        for g, name in enumerate(self.TIMING_GROUPS):
            ms, n = C.c_double(), C.c_int64()
            _check(lib().ddm_read_timing(self.ctx, g, C.byref(ms), C.byref(n)))
            out[name] = (ms.value, n.value)
        return out

    # -- diagnostics --------------------------------------------------------------
    DIAG_NAMES = ("mass", "momentum_x", "momentum_y", "momentum_z", "kinetic_energy", "case_tension",
                  "case_elastic", "case_projected", "clamps", "cfl", "grid_mass")

    def diagnostics(self) -> np.ndarray:
        """ddm_diagnostics: [n_inst, len(DIAG_NAMES)] float64 (host) for the
        current state: particle mass, momentum, kinetic energy, the return-map
        cases and clamps of the next constitutive update, the CFL number, and
        the grid mass of the last sub-step (NaN when there is none)."""
        t = self.torch
        out = t.empty((self.n_inst, len(self.DIAG_NAMES)), dtype=t.float64, device=self.device)
        self._inputs_ready()
        _check(lib().ddm_diagnostics(self.ctx, C.c_void_p(out.data_ptr())))
        self._outputs_ready()
        return out.cpu().numpy()

    def check(self) -> DdmDeviceError:
        e = DdmDeviceError()
        _check(lib().ddm_check(self.ctx, C.byref(e)))
        return e


# ---------------------------------------------------------------------------
# a batch on several streams
# ---------------------------------------------------------------------------

def balanced_groups(counts: Sequence[int], n_groups: int):
    """Instance indices in n_groups groups of near-equal particle count: the
    instances by decreasing count dealt out in snake order (0, 1, .., n-1,
    n-1, .., 0, ...); each group keeps its instances in their original order."""
    order = sorted(range(len(counts)), key=lambda i: -int(counts[i]))
    groups = [[] for _ in range(n_groups)]
    for k, i in enumerate(order):
        r = k % (2 * n_groups)
        groups[r if r < n_groups else 2 * n_groups - 1 - r].append(i)
    return [sorted(g) for g in groups if g]


class StreamGroup:
    """A batch run as several contexts at once: the instances split into
    groups (balanced_groups), one Simulator per group on a stream of its own.
    A pass issues every group's ddm_pass (graph-replayed by default) without
    waits between the streams, so one group's kernels fill the slots that
    another's leave idle (launch tails, the short grid kernels, binning).  The
    results are those of the groups' own contexts, returned in the original
    instance order; every kernel is the library's, and this class only splits
    the inputs and gathers the outputs."""

    def __init__(self, cfg: DdmConfig, instances: Sequence[DdmInstance], groups, record_segments=None,
                 grid_record_blocks=None, device="cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.instances = list(instances)
        self.n_inst = len(self.instances)
        self.groups = [list(g) for g in groups]
        assert sorted(i for g in self.groups for i in g) == list(range(self.n_inst)), "groups must partition"
        self.sims = []
        for k, g in enumerate(self.groups):
            c = DdmConfig.from_buffer_copy(cfg)
            if record_segments is not None:
                c.record_segments = int(record_segments[k])
            if grid_record_blocks is not None:
                c.grid_record_blocks = int(grid_record_blocks[k])
            self.sims.append(Simulator(c, [self.instances[i] for i in g], device=device,
                                       stream=torch.cuda.Stream(self.device)))
        counts = [int(s.n_particles) for s in self.instances]
        starts = np.concatenate([[0], np.cumsum(counts)])
        # rows of the concatenated positions of each group, in the group's order
        self._rows = [torch.as_tensor(np.concatenate([np.arange(starts[i], starts[i + 1]) for i in g]),
                                      device=self.device) for g in self.groups]
        self._inst = [torch.as_tensor(g, device=self.device) for g in self.groups]
        self.npix = self.sims[0].npix
        self.dim = self.sims[0].dim
        self.dtype = self.sims[0].dtype

    def set_inputs(self, x0, target, dloss=None):
        """Splits the batch's inputs into the groups' buffers: x0 [sum N_i,
        dim], target [n_inst, npix] and dloss [n_inst] (ones when None) in
        the original instance order, host or device; each group's stream
        waits for the current stream before it reads them."""
        t = self.torch
        cur = t.cuda.current_stream(self.device)
        x0 = t.as_tensor(x0, device=self.device).reshape(-1, self.dim).to(self.dtype)
        tg = t.as_tensor(target, device=self.device, dtype=t.float64).reshape(self.n_inst, self.npix)
        dl = (t.ones(self.n_inst, dtype=t.float64, device=self.device) if dloss is None
              else t.as_tensor(dloss, device=self.device, dtype=t.float64).reshape(-1))
        self._in = []
        for sim, rows, idx in zip(self.sims, self._rows, self._inst):
            sim.stream.wait_stream(cur)
            with t.cuda.stream(sim.stream):
                self._in.append((x0.index_select(0, rows), tg.index_select(0, idx), dl.index_select(0, idx)))

    def run(self, n: int, graph: bool = True):
        """Issues one pass of every group (init, recorded rollout, loss,
        backward) on its own stream, with the inputs of set_inputs, and
        returns at once.  Each group's stream first waits for the work
        queued so far on the current stream (a results() copy of the last
        outputs, which the new pass overwrites); successive calls with
        nothing queued between them keep each group behind its own previous
        pass only, so a group that finishes early starts its next pass while
        the others still run."""
        t = self.torch
        cur = t.cuda.current_stream(self.device)
        self._out = []
        for sim, (x0, tg, dl) in zip(self.sims, self._in):
            sim.stream.wait_stream(cur)
            with t.cuda.stream(sim.stream):
                self._out.append(sim.full_pass(x0, n, tg, dl, graph=graph))

    def join(self):
        """Makes the current stream wait for every group's last pass (no
        copies): with run(), one joined step of the whole batch."""
        cur = self.torch.cuda.current_stream(self.device)
        for sim in self.sims:
            cur.wait_stream(sim.stream)

    def results(self):
        """(loss [n_inst], grad [n_inst, N_PARAMS]) of the last run, in the
        original instance order, on the current stream."""
        t = self.torch
        cur = t.cuda.current_stream(self.device)
        loss = t.empty(self.n_inst, dtype=t.float64, device=self.device)
        grad = t.empty((self.n_inst, N_PARAMS), dtype=t.float64, device=self.device)
        for sim, idx, (l, g) in zip(self.sims, self._inst, self._out):
            cur.wait_stream(sim.stream)
            loss.index_copy_(0, idx, l)
            grad.index_copy_(0, idx, g)
        return loss, grad

    def full_pass(self, x0, n: int, target, dloss=None, graph: bool = True):
        """set_inputs, run and results in one call."""
        self.set_inputs(x0, target, dloss)
        self.run(n, graph=graph)
        return self.results()

    def check(self):
        """ddm_check of every group: the first failing group's error, else the
        (all-zero) error record of the first."""
        errs = [s.check() for s in self.sims]
        for e in errs:
            if e.flags:
                return e
        return errs[0]

    def synchronize(self):
        for s in self.sims:
            s.stream.synchronize()


# ---------------------------------------------------------------------------
# autograd
# ---------------------------------------------------------------------------

def _autograd_function():
    import torch

    class DigLoss(torch.autograd.Function):
        """loss[n_inst] = rollout + loss of the digging simulation; gradients with
        respect to params[n_inst, N_PARAMS] (PARAM_NAMES order) come from the
        library's reverse pass (checkpointed recompute)."""

        @staticmethod
        def forward(ctx, params, x0, target, cfg, instances, steps):
            p = params.detach().double().cpu().numpy()
            insts = []
            for i, base in enumerate(instances):
                s = DdmInstance()
                C.pointer(s)[0] = base
                (s.E, s.nu, s.phi_deg, s.rho, s.depth, s.angle_deg, s.push, s.displace,
                 s.push_angle_deg) = (float(v) for v in p[i])
                insts.append(s)
            on_gpu = isinstance(x0, torch.Tensor) and x0.is_cuda
            sim = Simulator(cfg, insts, device=x0.device if on_gpu else "cuda")
            sim.init_state(x0)
            sim.rollout(steps)
            loss = sim.loss(target)
            ctx.sim = sim
            ctx.param_device = params.device
            ctx.param_dtype = params.dtype
            return loss.to(params.device)

        @staticmethod
        def backward(ctx, grad_out):
            g = ctx.sim.backward(grad_out.detach().to(ctx.sim.device, torch.float64))
            return g.to(ctx.param_device, ctx.param_dtype), None, None, None, None, None

    return DigLoss


_DIGLOSS = None


def dig_loss(params, x0, target, cfg: DdmConfig, instances: Sequence[DdmInstance], steps: int):
    """Differentiable loss per instance; see DigLoss."""
    global _DIGLOSS
    if _DIGLOSS is None:
        _DIGLOSS = _autograd_function()
    return _DIGLOSS.apply(params, x0, target, cfg, list(instances), int(steps))
