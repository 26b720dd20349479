"""Brute-force GCDF of a small planar mobile manipulator (test infrastructure).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The robot: a planar base (x, y, yaw) carrying a disc body of radius 0.25 m
and a 2-link arm whose shoulder sits at the base centre; link 1 (length 0.6)
points at angle a1 from the base x axis, link 2 (length 0.5) at a1 + a2; each
link is a capsule of radius 0.05.  Its exact 2-D signed distance is the minimum
of the disc and capsule distances (exact outside the robot).

The GCDF (Definition 1) with M = diag(w_t, w_t, 1, 1, 1) over
(x, y, yaw, a1, a2) is the M-weighted distance from q to the set of
configurations whose surface passes through p.  For a fixed rotational part
(yaw', a') the cheapest translation that puts p on the surface moves the base
by exactly the workspace distance, so the translational cost is
w_t * sdf(R(yaw')^T (p - t); a')^2.  The search clamps sdf at zero, which makes
B the distance to the union of solid slices; where the minimiser has p strictly
outside the robot (sdf > 0, the only pairs the tests use) that minimiser lies
on the zero set and B is the distance to it.  Writing the yaw offset
phi = yaw' - yaw and p' = R(yaw)^T (p - t), the base-frame function is

    B(p', a)^2 = min_{phi, a'}  w_t * max(sdf(R(phi)^T p'; a'), 0)^2 + phi^2 + |wrap(a - a')|^2.

Revolute coordinates wrap (the zero set holds every 2*pi-periodic copy).

Search: a' on an absolute 48 x 48 grid over [-pi, pi)^2; phi continuous (a
64-point grid, golden-section refinement for the 16 best arm candidates, then
secant steps on the analytic derivative in phi).  With a' absolute and phi relative, B is an exact distance to a
union of continuous slices of the zero set, so the weighted eikonal property
(Theorem 1, part 1) holds exactly where B is differentiable, and B is exactly
invariant to a common rigid motion of base and point.

The gradient of B is taken at the minimiser (envelope theorem), which equals
the closed form grad f = M (q - q_z) / f of the proof of Theorem 1.
"""
from __future__ import annotations

import math

import numpy as np

R_BODY = 0.25
L1, L2 = 0.6, 0.5
R_LINK = 0.05
N_ARM_GRID = 48
N_PHI_GRID = 64
N_REFINE = 16


def wrap(a):
    """Wrap angles to [-pi, pi)."""
    return (np.asarray(a) + math.pi) % (2.0 * math.pi) - math.pi


def _seg_dist(px, py, ax, ay, bx, by):
    """Distance from points to segments a-b and the closest point (broadcasting)."""
    dx, dy = bx - ax, by - ay
    ll = dx * dx + dy * dy
    t = np.clip(((px - ax) * dx + (py - ay) * dy) / ll, 0.0, 1.0)
    cx, cy = ax + t * dx, ay + t * dy
    return np.hypot(px - cx, py - cy), cx, cy


def sdf_base(px, py, a1, a2, with_grad: bool = False):
    """Signed distance of base-frame point (px, py) to the robot with arm (a1, a2).

    Returns sdf (and d sdf / d(px, py) if with_grad), broadcasting over inputs.
    """
    px, py, a1, a2 = np.broadcast_arrays(*(np.asarray(v, dtype=np.float64) for v in (px, py, a1, a2)))
    ex, ey = L1 * np.cos(a1), L1 * np.sin(a1)
    wx, wy = ex + L2 * np.cos(a1 + a2), ey + L2 * np.sin(a1 + a2)
    zero = np.zeros_like(px)
    d0 = np.hypot(px, py)
    s0 = d0 - R_BODY
    d1, c1x, c1y = _seg_dist(px, py, zero, zero, ex, ey)
    s1 = d1 - R_LINK
    d2, c2x, c2y = _seg_dist(px, py, ex, ey, wx, wy)
    s2 = d2 - R_LINK
    s = np.minimum(np.minimum(s0, s1), s2)
    if not with_grad:
        return s
    # gradient of the active piece: unit vector from its closest point to p
    gx = np.where(s == s0, px / d0, np.where(s == s1, (px - c1x) / d1, (px - c2x) / d2))
    gy = np.where(s == s0, py / d0, np.where(s == s1, (py - c1y) / d1, (py - c2y) / d2))
    return s, gx, gy


def sdf_world(p, q):
    """Signed distance of world point p (x, y) to the robot at configuration q (x, y, yaw, a1, a2)."""
    c, s = math.cos(q[2]), math.sin(q[2])
    ux, uy = p[0] - q[0], p[1] - q[1]
    return float(sdf_base(c * ux + s * uy, -s * ux + c * uy, q[3], q[4]))


def _rot_t(phi, px, py):
    """R(phi)^T applied to (px, py)."""
    c, s = np.cos(phi), np.sin(phi)
    return c * px + s * py, -s * px + c * py


def _cost(phi, px, py, a1g, a2g, da2, w_t):
    rx, ry = _rot_t(phi, px, py)
    sd = np.maximum(sdf_base(rx, ry, a1g, a2g), 0.0)
    return w_t * sd * sd + phi * phi + da2


def _dcost_dphi(phi, px, py, a1g, a2g, w_t):
    """d/dphi of the cost: 2 w_t sdf+ (grad sdf . d(R(phi)^T p')/dphi) + 2 phi."""
    rx, ry = _rot_t(phi, px, py)
    s, gx, gy = sdf_base(rx, ry, a1g, a2g, with_grad=True)
    return float(2.0 * w_t * max(float(s), 0.0) * (gx * ry - gy * rx) + 2.0 * phi)


def _polish_phi(phi, px, py, a1g, a2g, w_t):
    """Secant iterations on the cost derivative: golden section alone resolves a
    quadratic minimum only to about sqrt(machine epsilon)."""
    x0, x1 = phi - 1e-7, phi + 1e-7
    f0 = _dcost_dphi(x0, px, py, a1g, a2g, w_t)
    f1 = _dcost_dphi(x1, px, py, a1g, a2g, w_t)
    for _ in range(30):
        if f1 == f0:
            break
        x2 = x1 - f1 * (x1 - x0) / (f1 - f0)
        if abs(x2 - phi) > 1e-3:  # left the local basin: keep the bracketed value
            return phi
        x0, f0 = x1, f1
        x1 = x2
        f1 = _dcost_dphi(x1, px, py, a1g, a2g, w_t)
        if abs(x1 - x0) < 1e-16:
            break
    return x1


def gcdf_base(pxy, a, w_t: float = 1.0, tol: float = 1e-12):
    """B(p', a) for one base-frame point (p'x, p'y) and arm (a1, a2).

    Returns dict with: value B, e = dB/d(p'x, p'y, a1, a2), the minimiser
    (phi, a1', a2'), the signed distance at the minimiser, and ``gap`` = the
    relative gap between the best and second-best arm candidates (small gap:
    the gradient may not be unique).
    """
    px, py = float(pxy[0]), float(pxy[1])
    grid = -math.pi + 2.0 * math.pi * np.arange(N_ARM_GRID) / N_ARM_GRID
    A1, A2 = np.meshgrid(grid, grid, indexing="ij")
    A1, A2 = A1.ravel(), A2.ravel()
    da2 = wrap(a[0] - A1) ** 2 + wrap(a[1] - A2) ** 2
    phis = -math.pi + 2.0 * math.pi * np.arange(N_PHI_GRID) / N_PHI_GRID
    C = _cost(phis[:, None], px, py, A1[None, :], A2[None, :], da2[None, :], w_t)  # (phi, arm)
    best_phi_idx = np.argmin(C, axis=0)
    best_c = C[best_phi_idx, np.arange(len(A1))]
    cand = np.argsort(best_c)[:N_REFINE]
    h = 2.0 * math.pi / N_PHI_GRID
    gr = (math.sqrt(5.0) - 1.0) / 2.0
    results = []
    for ci in cand:
        lo = phis[best_phi_idx[ci]] - h
        hi = phis[best_phi_idx[ci]] + h
        f = lambda ph: float(_cost(ph, px, py, A1[ci], A2[ci], da2[ci], w_t))
        x1, x2 = hi - gr * (hi - lo), lo + gr * (hi - lo)
        f1, f2 = f(x1), f(x2)
        while hi - lo > tol:
            if f1 < f2:
                hi, x2, f2 = x2, x1, f1
                x1 = hi - gr * (hi - lo)
                f1 = f(x1)
            else:
                lo, x1, f1 = x1, x2, f2
                x2 = lo + gr * (hi - lo)
                f2 = f(x2)
        ph = _polish_phi(0.5 * (lo + hi), px, py, A1[ci], A2[ci], w_t)
        results.append((f(ph), ph, ci))
    results.sort()
    c2, phi, ci = results[0]
    gap = (results[1][0] - c2) / max(c2, 1e-300) if len(results) > 1 else np.inf
    B = math.sqrt(c2)
    a1p, a2p = A1[ci], A2[ci]
    rx, ry = _rot_t(phi, px, py)
    s, gx, gy = sdf_base(rx, ry, a1p, a2p, with_grad=True)
    s, gx, gy = float(s), float(gx), float(gy)
    sp = max(s, 0.0)
    # d(sdf(R(phi)^T p'))/dp' = R(phi) grad sdf
    c, sn = math.cos(phi), math.sin(phi)
    gpx, gpy = c * gx - sn * gy, sn * gx + c * gy
    e = np.array([w_t * sp * gpx / B, w_t * sp * gpy / B,
                  float(wrap(a[0] - a1p)) / B, float(wrap(a[1] - a2p)) / B])
    return {"value": B, "e": e, "phi": phi, "arm": (float(a1p), float(a2p)), "sdf": s, "gap": gap}


def gcdf_value(pxy, a, w_t: float = 1.0) -> float:
    return gcdf_base(pxy, a, w_t)["value"]
