"""ctypes front end of the FP64 oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It compiles ``oracle.cpp`` with g++ (no
fast-math, no FP contraction) into ``liboracle.so`` next to it and wraps the C
interface with numpy arrays.  The product path never touches it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))

# Differentiable inputs, in the order of rollout's params and gradient:
# E, nu, phi_deg, rho, depth, angle_deg, push, displace, push_angle_deg.
N_PARAMS = 9
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = [os.path.join(_HERE, "oracle.cpp"), os.path.join(_HERE, "dual.hpp"), os.path.join(_HERE, "tape.hpp")]


def build(force: bool = True) -> str:
    """Compile the oracle.  -O2, -ffp-contract=off, no fast-math, single thread."""
    if not force and os.path.exists(LIB_PATH) and all(
            os.path.getmtime(LIB_PATH) >= os.path.getmtime(s) for s in _SRC):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-o", tmp, _SRC[0], "-lquadmath"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class OrcConfig(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("n_grid", C.c_int32), ("bound", C.c_int32), ("n_sub", C.c_int32),
        ("shovel", C.c_int32), ("hm_res", C.c_int32), ("region_sign", C.c_int32), ("skill_unrounded", C.c_int32),
        ("dt", C.c_double), ("gravity", C.c_double), ("ppc", C.c_double),
        ("half_w", C.c_double), ("half_n", C.c_double), ("half_p", C.c_double),
        ("skin", C.c_double), ("mu_b", C.c_double),
        ("v_l", C.c_double), ("v_w", C.c_double), ("d_lift", C.c_double),
        ("tip0", C.c_double * 3),
        ("hm_origin", C.c_double * 2), ("hm_size", C.c_double), ("hm_offset", C.c_double),
        ("region_depth", C.c_double), ("m_target", C.c_double), ("m_ref", C.c_double),
        ("w_mass", C.c_double), ("w_hm", C.c_double),
        ("cohesion", C.c_double),
        ("particle_contact", C.c_int32), ("pad1", C.c_int32),
        ("w_emd", C.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.orc_rollout.restype = C.c_int
        L.orc_rollout.argtypes = [C.POINTER(OrcConfig), dp, C.c_int, dp, C.c_int, C.c_int, dp, dp, dp, dp, dp,
                                  C.POINTER(C.c_int64), dp, dp, C.c_int]
        L.orc_rollout_reverse.restype = C.c_int
        L.orc_rollout_reverse.argtypes = [C.POINTER(OrcConfig), dp, C.c_int, dp, C.c_int, C.c_int, dp, C.c_int,
                                          C.c_double, C.c_double, C.c_double, dp, dp, dp]
        L.orc_treat.restype = None
        L.orc_treat.argtypes = [C.c_int, C.c_int, dp, C.c_double, C.c_double, C.c_double]
        L.orc_assign.restype = C.c_int
        L.orc_assign.argtypes = [C.c_int, C.c_int, dp, C.POINTER(C.c_int)]
        L.orc_diagnostics.restype = C.c_int
        L.orc_diagnostics.argtypes = [C.POINTER(OrcConfig), dp, C.c_int, dp, dp]
        L.orc_heightmap.restype = C.c_int
        L.orc_heightmap.argtypes = [C.POINTER(OrcConfig), C.c_int, dp, dp, C.POINTER(C.c_int)]
        L.orc_surface_particles.restype = C.c_int
        L.orc_surface_particles.argtypes = [C.POINTER(OrcConfig), C.c_int, dp, C.POINTER(C.c_int)]
        L.orc_skill_actions.restype = C.c_int
        L.orc_skill_actions.argtypes = [dp, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int, C.c_int,
                                        C.POINTER(C.c_int), dp, dp]
        L.orc_pose_table.restype = C.c_int
        L.orc_pose_table.argtypes = [C.POINTER(OrcConfig), dp, C.c_double, C.c_int, dp, dp]
        L.orc_svd.argtypes = [C.c_int, dp, dp, dp, dp]
        L.orc_material.argtypes = [C.c_double] * 4 + [dp]
        L.orc_material.restype = None
        L.orc_return_map.restype = C.c_int
        L.orc_return_map.argtypes = [C.c_int, dp, C.c_double, C.c_double, C.c_double, C.c_double, dp, dp]
        L.orc_delta_gamma.restype = C.c_double
        L.orc_delta_gamma.argtypes = [C.c_int, dp, C.c_double, C.c_double, C.c_double, C.c_double]
        L.orc_constitutive.restype = C.c_int
        L.orc_constitutive.argtypes = [C.c_int, dp, C.c_double, C.c_double, C.c_double, C.c_double,
                                       dp, dp, dp, dp, dp, dp]
        L.orc_box_sdf.restype = C.c_double
        L.orc_box_sdf.argtypes = [C.POINTER(OrcConfig), dp, C.c_double, dp, dp]
        L.orc_coulomb.restype = None
        L.orc_coulomb.argtypes = [dp, dp, C.c_double, dp]
        L.orc_bin.restype = C.c_int
        L.orc_bin.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, dp, C.POINTER(C.c_int32),
                              C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def config(w, shovel: Optional[bool] = None, **over) -> OrcConfig:
    """Oracle configuration from a workloads.Workload (same numbers the GPU gets)."""
    c = OrcConfig()
    c.dim, c.n_grid, c.bound, c.n_sub = w.dim, w.n_grid, w.bound, w.n_sub
    c.shovel = int(w.skill is not None if shovel is None else shovel)
    c.hm_res, c.region_sign = w.hm_res, w.region_sign
    c.dt, c.gravity, c.ppc = w.dt, w.gravity, float(w.ppc)
    c.half_w, c.half_n, c.half_p = w.shovel_half
    c.skin, c.mu_b = w.skin, w.mu_b
    c.v_l, c.v_w, c.d_lift = w.v_l, w.v_w, w.d_lift
    t = list(w.tip0) + [0.0] * (3 - w.dim)
    for k in range(3):
        c.tip0[k] = t[k]
    c.hm_origin[0], c.hm_origin[1] = w.hm_origin
    c.hm_size, c.hm_offset = w.hm_size, w.hm_offset
    c.region_depth, c.m_target, c.m_ref = w.region_depth, w.m_target, w.m_ref
    c.w_mass, c.w_hm = w.w_mass, w.w_hm
    c.cohesion = w.material.cohesion
    c.skill_unrounded = int(w.skill_unrounded)
    c.particle_contact = int(w.particle_contact)
    c.w_emd = float(getattr(w, "w_emd", 0.0))
    for k, v in over.items():
        setattr(c, k, v)
    return c


def state_size(dim: int) -> int:
    return 2 * dim + 2 * dim * dim


def initial_state(x0: np.ndarray) -> np.ndarray:
    """Packed per-particle state [x, v, C, F] with v = 0, C = 0, F = I."""
    n, d = x0.shape
    s = np.zeros((n, state_size(d)), dtype=np.float64)
    s[:, :d] = x0
    s[:, 2 * d + d * d:] = np.eye(d).reshape(-1)
    return s


def unpack(state: np.ndarray, d: int):
    n = state.shape[0]
    x = state[:, :d]
    v = state[:, d:2 * d]
    Cm = state[:, 2 * d:2 * d + d * d].reshape(n, d, d)
    F = state[:, 2 * d + d * d:].reshape(n, d, d)
    return x, v, Cm, F


class OracleError(RuntimeError):
    pass


def rollout(cfg: OrcConfig, params: np.ndarray, state: np.ndarray, n_steps: int, step0: int = 0,
            target: Optional[np.ndarray] = None, grad: bool = False, want_grid: bool = False,
            emd_target: Optional[np.ndarray] = None):
    """Run sub-steps [step0, step0+n_steps).  Returns a dict with the final state,
    and loss / grad / height map when a target is given, grid of the last step
    (m, mv[3], v[3] per node) when asked."""
    L = lib()
    state = np.ascontiguousarray(state, dtype=np.float64)
    params = np.ascontiguousarray(params, dtype=np.float64)
    n = state.shape[0]
    out = np.zeros_like(state)
    loss = np.zeros(1)
    g = np.zeros(N_PARAMS) if grad else None
    npix = cfg.hm_res ** (cfg.dim - 1)
    hm = np.zeros(npix) if target is not None else None
    tgt = np.ascontiguousarray(target, dtype=np.float64).reshape(-1) if target is not None else None
    stats = np.zeros(8, dtype=np.int64)
    nodes = cfg.n_grid ** cfg.dim
    grid = np.zeros((nodes, 7)) if want_grid else None
    et = np.ascontiguousarray(emd_target, dtype=np.float64).reshape(-1, 3) if emd_target is not None else None
    rc = L.orc_rollout(C.byref(cfg), _p(params), n, _p(state), step0, n_steps, _p(out), _p(tgt), _p(loss),
                       _p(g), _p(hm), stats.ctypes.data_as(C.POINTER(C.c_int64)), _p(grid), _p(et),
                       0 if et is None else et.shape[0])
    if rc != 0:
        raise OracleError(f"oracle rollout failed with code {rc} (stats {stats.tolist()})")
    res = {"state": out, "stats": stats}
    if target is not None:
        res["loss"] = float(loss[0])
        res["heightmap"] = hm
    if grad:
        res["grad"] = g
    if want_grid:
        res["grid"] = grid
    return res


TREAT_MODES = ("none", "clip", "scale", "norm")


def rollout_reverse(cfg: OrcConfig, params: np.ndarray, state: np.ndarray, n_steps: int, target: np.ndarray,
                    step0: int = 0, mode: str = "none", clip: float = 1e4, oom: float = 4.0, delta: float = 1e-6,
                    stats: bool = False):
    """Reverse-mode (tape) gradient of the loss after sub-steps [step0,
    step0 + n_steps), with the gradient treatment `mode` of Sec. III-E inside
    the adjoint sweep.  Returns {"loss", "grad" [9], and "stats"
    [n_steps, 6, 6] when asked: per sub-step and variable (x, v, F, grid v,
    grid mv, grid m) the max, min, 2-norm before and after the treatment}."""
    state = np.ascontiguousarray(state, dtype=np.float64)
    params = np.ascontiguousarray(params, dtype=np.float64)
    tgt = np.ascontiguousarray(target, dtype=np.float64).reshape(-1)
    loss = np.zeros(1)
    g = np.zeros(N_PARAMS)
    st = np.zeros((n_steps, 6, 6)) if stats else None
    rc = lib().orc_rollout_reverse(C.byref(cfg), _p(params), state.shape[0], _p(state), step0, n_steps, _p(tgt),
                                   TREAT_MODES.index(mode), clip, oom, delta, _p(loss), _p(g), _p(st))
    if rc != 0:
        raise OracleError(f"reverse rollout failed with code {rc}")
    out = {"loss": float(loss[0]), "grad": g}
    if stats:
        out["stats"] = st
    return out


def treat(g: np.ndarray, mode: str, clip: float = 1e4, oom: float = 4.0, delta: float = 1e-6) -> np.ndarray:
    """The C++ oracle's treatment of one vector (orc_treat)."""
    g = np.array(g, dtype=np.float64).ravel()
    lib().orc_treat(TREAT_MODES.index(mode), g.size, _p(g), clip, oom, delta)
    return g


def skill_actions(theta, v_l=3.0, v_w=10.0 * np.pi, dta=2e-3, d4=0.01, max_T=10000, unrounded=False):
    L = lib()
    th = np.ascontiguousarray(theta, dtype=np.float64)
    T = (C.c_int * 4)()
    acts = np.zeros((max_T, 6))
    jac = np.zeros((max_T, 6, 5))
    n = L.orc_skill_actions(_p(th), v_l, v_w, dta, d4, int(bool(unrounded)), max_T, T, _p(acts), _p(jac))
    if n < 0:
        raise OracleError("too many actions")
    return list(T), acts[:n].copy(), jac[:n].copy()


def pose_table(cfg: OrcConfig, skill5, dt: float, n_steps: int):
    """Pose rows and their Jacobian [n_steps, 8, 5] with respect to the
    physical skill parameters (depth, angle_deg, push, displace, push_angle_deg)."""
    sk = np.ascontiguousarray(skill5, dtype=np.float64)
    out = np.zeros((n_steps, 8))
    jac = np.zeros((n_steps, 8, 5))
    lib().orc_pose_table(C.byref(cfg), _p(sk), dt, n_steps, _p(out), _p(jac))
    return out, jac


def svd(F: np.ndarray):
    d = F.shape[0]
    F = np.ascontiguousarray(F, dtype=np.float64)
    U, S, V = np.zeros((d, d)), np.zeros(3), np.zeros((d, d))
    lib().orc_svd(d, _p(F), _p(U), _p(S), _p(V))
    return U, S[:d].copy(), V


def material(E, nu, phi_deg, cohesion=0.0):
    out = np.zeros(4)
    lib().orc_material(E, nu, phi_deg, cohesion, _p(out))
    return tuple(out)      # mu, lambda, alpha_f, k_c


def return_map(d, s, mu, lam, alpha, kc=0.0):
    s3 = np.ones(3)
    s3[:d] = s
    g, h = np.zeros(3), np.zeros(3)
    cs = lib().orc_return_map(d, _p(s3), mu, lam, alpha, kc, _p(g), _p(h))
    return cs, g[:d].copy(), h[:d].copy()


def delta_gamma(d, s, mu, lam, alpha, kc=0.0):
    s3 = np.ones(3)
    s3[:d] = s
    return lib().orc_delta_gamma(d, _p(s3), mu, lam, alpha, kc)


def constitutive(Ft, E, nu, phi_deg, cohesion=0.0, dFt=None, dpar=None):
    d = Ft.shape[0]
    Ft = np.ascontiguousarray(Ft, dtype=np.float64)
    dFt = None if dFt is None else np.ascontiguousarray(dFt, dtype=np.float64)
    dpar = None if dpar is None else np.ascontiguousarray(dpar, dtype=np.float64)
    Fn, tau, dFn, dtau = (np.zeros((d, d)) for _ in range(4))
    cs = lib().orc_constitutive(d, _p(Ft), E, nu, phi_deg, cohesion, _p(dFt), _p(dpar), _p(Fn), _p(tau),
                                _p(dFn), _p(dtau))
    return cs, Fn, tau, dFn, dtau


def box_sdf(cfg: OrcConfig, tip, psi, x):
    n = np.zeros(3)
    phi = lib().orc_box_sdf(C.byref(cfg), _p(np.asarray(tip, dtype=np.float64)), psi,
                            _p(np.asarray(x, dtype=np.float64)), _p(n))
    return phi, n


def coulomb(vs, n, mu_b, v):
    v = np.array(v, dtype=np.float64)
    lib().orc_coulomb(_p(np.asarray(vs, dtype=np.float64)), _p(np.asarray(n, dtype=np.float64)), mu_b, _p(v))
    return v


def bin_keys(x: np.ndarray, n_grid: int, tile: int, inst: Optional[np.ndarray] = None):
    x = np.ascontiguousarray(x, dtype=np.float64)
    n, d = x.shape
    keys = np.zeros(n, dtype=np.uint32)
    perm = np.zeros(n, dtype=np.uint32)
    ip = None
    if inst is not None:
        inst = np.ascontiguousarray(inst, dtype=np.int32)
        ip = inst.ctypes.data_as(C.POINTER(C.c_int32))
    rc = lib().orc_bin(n, d, n_grid, tile, _p(x), ip, keys.ctypes.data_as(C.POINTER(C.c_uint32)),
                       perm.ctypes.data_as(C.POINTER(C.c_uint32)))
    if rc != 0:
        raise OracleError(f"binning failed with code {rc}")
    return keys, perm


def assign(cost: np.ndarray) -> np.ndarray:
    """Column of every row of the cheapest one-to-one assignment (rows <= columns)."""
    cost = np.ascontiguousarray(cost, dtype=np.float64)
    n, m = cost.shape
    out = np.zeros(n, dtype=np.int32)
    if lib().orc_assign(n, m, _p(cost), out.ctypes.data_as(C.POINTER(C.c_int))) != 0:
        raise OracleError("bad assignment shape")
    return out


def surface_particles(cfg: OrcConfig, state: np.ndarray) -> np.ndarray:
    """Indices of the particles of the surface observation, in pixel order."""
    state = np.ascontiguousarray(state, dtype=np.float64)
    out = np.zeros(cfg.hm_res ** 2, dtype=np.int32)
    n = lib().orc_surface_particles(C.byref(cfg), state.shape[0], _p(state), out.ctypes.data_as(C.POINTER(C.c_int)))
    return out[:n].copy()


def heightmap(cfg: OrcConfig, state: np.ndarray):
    """Height map of Eq. hm for the positions of a packed state, and the owner
    (particle index, -1 when empty) of every pixel."""
    state = np.ascontiguousarray(state, dtype=np.float64)
    npix = cfg.hm_res ** (cfg.dim - 1)
    hm = np.zeros(npix)
    own = np.zeros(npix, dtype=np.int32)
    lib().orc_heightmap(C.byref(cfg), state.shape[0], _p(state), _p(hm), own.ctypes.data_as(C.POINTER(C.c_int)))
    return hm, own


DIAG_NAMES = ("mass", "momentum_x", "momentum_y", "momentum_z", "kinetic_energy", "case_tension", "case_elastic",
              "case_projected", "clamps", "cfl", "grid_mass")


def diagnostics(cfg: OrcConfig, params: np.ndarray, state: np.ndarray) -> np.ndarray:
    """Diagnostics of a packed state (DIAG_NAMES): mass, momentum, kinetic
    energy, the return-map cases and clamps of the next constitutive update,
    the CFL number; the grid mass entry is NaN (it needs the last sub-step's
    grid: sum the masses of rollout(..., grid=True))."""
    state = np.ascontiguousarray(state, dtype=np.float64)
    out = np.zeros(len(DIAG_NAMES))
    rc = lib().orc_diagnostics(C.byref(cfg), _p(np.asarray(params, dtype=np.float64)), state.shape[0], _p(state),
                               _p(out))
    if rc != 0:
        raise ValueError(f"orc_diagnostics failed ({rc})")
    return out
