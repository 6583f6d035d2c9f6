"""Brute-force pins of the oracle's loss (Sec. III-A "Goal", Eq. hm, and the
scoop-mass term).

The height map, its pixel owners and the scoop-region mass are recomputed here
in numpy from their definitions, written independently of the oracle's loops:
  * height map: every particle marks the pixels of its own (x, z) and of the
    four points r_p away along x and z (2D: x and x +- r_p); a pixel holds the
    largest height y that reaches it, 0 when none above 0 does, and its owner
    is the lowest-numbered particle at that height; points outside the window
    are dropped;
  * scoop mass: M_in = sum over grid nodes inside the slab in front of the
    final blade pose of the node mass sum_p N(x_p - x_i) m_p, with the
    quadratic B-spline kernel N evaluated as a function of distance (not the
    base-cell form the method uses);
  * loss = w_hm / n_pix * sum(((H - H_target) / dx)^2) + w_mass ((M_in - M*) / M_ref)^2.
CPU only.
"""
import numpy as np
import pytest

import workloads as W


def bspline(r):
    """Quadratic B-spline kernel of the distance in cells."""
    a = np.abs(r)
    return np.where(a < 0.5, 0.75 - a * a, np.where(a < 1.5, 0.5 * (1.5 - a) ** 2, 0.0))


def brute_heightmap(w, x):
    d, res = w.dim, w.hm_res
    pix = w.hm_size / res
    r = w.hm_offset
    offs = [(0, 0), (r, 0), (-r, 0), (0, r), (0, -r)] if d == 3 else [(0, 0), (r, 0), (-r, 0)]
    H = np.zeros(res ** (d - 1))
    own = np.full(res ** (d - 1), -1)
    marks = {}                                   # pixel -> list of particles reaching it
    for p in range(x.shape[0]):
        for ox, oz in offs:
            ix = int(np.floor((x[p, 0] + ox - w.hm_origin[0]) / pix))
            if not 0 <= ix < res:
                continue
            if d == 3:
                iz = int(np.floor((x[p, 2] + oz - w.hm_origin[1]) / pix))
                if not 0 <= iz < res:
                    continue
                key = ix * res + iz
            else:
                key = ix
            marks.setdefault(key, set()).add(p)
    for key, ps in marks.items():
        ps = sorted(ps)
        ys = x[ps, 1]
        top = ys.max()
        if top > 0.0:
            H[key] = top
            own[key] = ps[int(np.argmax(ys == top))]
    return H, own


def blade_frame(tip, psi, half_p):
    e_w = np.array([0.0, 0.0, 1.0])
    e_n = np.array([np.cos(psi), -np.sin(psi), 0.0])
    e_p = np.array([-np.sin(psi), -np.cos(psi), 0.0])
    return tip - half_p * e_p, (e_w, e_n, e_p)


def brute_scoop_mass(w, x, tip, psi):
    dx = w.dx
    centre, (e_w, e_n, e_p) = blade_frame(np.asarray(tip), psi, w.shovel_half[2])
    mp = w.material.rho * dx ** 3 / w.ppc
    total = 0.0
    for p in range(x.shape[0]):
        lo = np.floor(x[p] / dx).astype(int) - 1
        grids = np.stack(np.meshgrid(*[np.arange(lo[a], lo[a] + 4) for a in range(3)], indexing="ij"),
                         -1).reshape(-1, 3)
        wts = np.prod(bspline(x[p][None, :] / dx - grids), axis=1)
        xi = grids * dx - centre[None, :]
        qw, qn, qp = xi @ e_w, xi @ e_n, xi @ e_p
        sn = w.region_sign * qn
        inside = ((np.abs(qw) <= w.shovel_half[0]) & (np.abs(qp) <= w.shovel_half[2])
                  & (sn > w.shovel_half[1]) & (sn <= w.shovel_half[1] + w.region_depth))
        total += mp * wts[inside].sum()
    return total


def _state(x, d):
    import oracle
    return oracle.initial_state(x)


def _scattered_state(w, n, seed, ties):
    """Random particles over the height-map window and beyond it, some sharing
    a height inside one pixel (ties), some at the window edges."""
    rng = np.random.default_rng(seed)
    d = w.dim
    lo = np.array([0.15, 0.1, 0.15])[:d] if d == 3 else np.array([0.15, 0.1])
    hi = np.array([0.85, 0.45, 0.85])[:d] if d == 3 else np.array([0.85, 0.45])
    x = lo + (hi - lo) * rng.random((n, d))
    pix = w.hm_size / w.hm_res
    if ties:
        # particles 3k, 3k+1, 3k+2 at one height in one pixel, numbered out of order
        for k in range(8):
            base = x[3 * k].copy()
            for j in (1, 2):
                x[3 * k + j] = base
                x[3 * k + j, 0] += (j * 0.2) * pix * (1 if base[0] < 0.5 else -1)
            x[3 * k + 2, 1] = x[3 * k, 1]
        # exact pixel edges of the window and just outside it
        x[30, 0] = w.hm_origin[0]
        x[31, 0] = w.hm_origin[0] + w.hm_size
        x[32, 0] = w.hm_origin[0] - 1e-12
        if d == 3:
            x[33, 2] = w.hm_origin[1] + 7 * pix
    return x


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("ties", [False, True])
def test_heightmap_brute_force(orc, d, ties):
    w = W.tiny(d, n_grid=64, shovel=(d == 3))
    x = _scattered_state(w, 300, 11 + d, ties)
    H, own = orc.heightmap(orc.config(w), orc.initial_state(x))
    Hb, ownb = brute_heightmap(w, x)
    assert np.array_equal(H, Hb)
    assert np.array_equal(own, ownb)
    assert (own < 0).any() and (own >= 0).any()      # both empty and filled pixels occur


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("terms", ["both", "height", "mass"])
@pytest.mark.parametrize("sign", [-1, 1])
def test_loss_brute_force(orc, d, terms, sign):
    """The loss of a scattered state after a step count that puts the blade in
    the bed (pose from the oracle's pose table, itself pinned to the paper's
    closed forms), against the brute-force height map and scoop mass."""
    w = W.tiny(d, n_grid=64, shovel=(d == 3))
    w.region_sign = sign
    if terms == "height":
        w.w_mass = 0.0
    elif terms == "mass":
        w.w_hm = 0.0
    rng = np.random.default_rng(5 + d)
    x = _scattered_state(w, 200, 21 + d, True)
    step = 157                                           # inside the push phase
    cfg = orc.config(w)
    if d == 3:
        pose, _ = orc.pose_table(cfg, w.params[4:], w.dt, step)
        tip, psi = pose[step - 1, :3], pose[step - 1, 3]
        # a cloud of particles around the slab in front of the blade, so that M_in > 0
        centre, (e_w, e_n, e_p) = blade_frame(tip, psi, w.shovel_half[2])
        u = rng.random((120, 3)) * 2 - 1
        q = centre[None, :] + (u[:, :1] * 0.06) * e_w + (u[:, 1:2] * 0.05) * e_n + (u[:, 2:] * 0.05) * e_p
        x = np.concatenate([x, q])
    target = np.asarray(W.target_heightmap(w, seed=9)).reshape(-1)
    r = orc.rollout(cfg, w.params, orc.initial_state(x), 0, step0=step, target=target)
    Hb, _ = brute_heightmap(w, x)
    npix = w.hm_res ** (d - 1)
    L = w.w_hm / npix * np.sum(((Hb - target) / w.dx) ** 2)
    if d == 3 and w.w_mass != 0.0:
        M = brute_scoop_mass(w, x, tip, psi)
        assert M > 0.0
        L += w.w_mass * ((M - w.m_target) / w.m_ref) ** 2
    np.testing.assert_array_equal(r["heightmap"], Hb)
    assert abs(r["loss"] - L) <= 1e-12 * abs(L), (r["loss"], L)
