"""Obstacle partitions and the sparse GCDF constraint Jacobian (test infrastructure).

TEST INFRASTRUCTURE ONLY, like the rest of this package: the tests, the smoke
check and the benchmark's CPU-baseline leg may call it; the product path never
does, and nothing here imports the product package.

Sec. IV-A (trajectory optimisation) of the paper:

* the obstacle set I_M is split into N overlapping partitions I_{M,i}, one per
  time step, holding the points within a range of the reference base
  position of that step;
* the GCDF constraints are stacked knot by knot into the dense vector c_gcdf
  of length m_1 + ... + m_N (eq. cdf_constraints_vector);
* the dense gradient rows of knot i (m_i x n) are mapped into the sparse
  (sum m_i) x 2Nn Jacobian by the projection matrices P_i, which place I_n
  at the columns of q_i inside the state x_i = [q_i, v_i] (eq.
  cdf_jacobian_construction).

Readings where the paper is silent or garbled:

* the partition's range (the paper leaves its metric open): planar Euclidean
  distance between the point's
  (x, y) and the reference base position, <= radius (z ignored).  The
  decision is taken in float32 exactly as written, dx*dx + dy*dy <= r*r with
  every operation rounded (no fused multiply-add), points in ascending
  index order inside a partition;
* sphere obstacles (x, y, z, s) of the primitive-aware extension (Sec. VII):
  the sphere is in range when it reaches into the disc, i.e. its centre's
  planar distance is <= radius + s, decided as dx*dx + dy*dy <= t*t with
  t = radius + s, every operation rounded in float32;
* the column offset of P_i prints as 2Nn(i-1), which overruns the matrix for
  i >= 2; the state layout x_i in R^{2n} puts q_i at columns 2n(i-1) + 1 ...
  2n(i-1) + n (1-based), which is the offset used here.
"""
from __future__ import annotations

import numpy as np

from . import eval_grad, eval_pairs

N_CONF = 9  # (x, y, yaw, a1..a6)


def partition(ref_xy, points, radius: float):
    """Brute-force partitions: for each reference base position, the indices of
    the points whose planar distance to it is within ``radius`` (for spheres,
    within ``radius`` plus the sphere's radius).

    ref_xy: (N, 2) base positions; points: (M, 3), or (M, 4) spheres.  Returns
    (offsets int64 (N+1,), idx int32 (sum m_i,)) in CSR form, ascending inside
    each row.
    """
    ref = np.asarray(ref_xy, np.float32).reshape(-1, 2)
    p = np.asarray(points, np.float32)
    if p.ndim != 2 or p.shape[1] not in (3, 4):
        raise ValueError("points must be (M, 3) or (M, 4)")
    if p.shape[1] == 4:
        t = np.float32(radius) + p[:, 3]
        r2 = t * t  # per sphere, float32
    else:
        r2 = np.float32(radius) * np.float32(radius)
    offsets = [0]
    idx = []
    for i in range(len(ref)):
        dx = p[:, 0] - ref[i, 0]
        dy = p[:, 1] - ref[i, 1]
        s = dx * dx + dy * dy  # float32, each product and the sum rounded
        sel = np.nonzero(s <= r2)[0]
        idx.append(sel)
        offsets.append(offsets[-1] + len(sel))
    idx = np.concatenate(idx).astype(np.int32) if idx else np.zeros(0, np.int32)
    return np.asarray(offsets, np.int64), idx


def row_knots(offsets):
    """Knot index of every stacked constraint row."""
    off = np.asarray(offsets, np.int64)
    return np.repeat(np.arange(len(off) - 1, dtype=np.int64), np.diff(off))


def constraints(blob: bytes, knots, points, offsets, idx):
    """c_gcdf (sum m_i,) and its dense gradient rows (sum m_i, n), float64:
    row r belongs to knot i = row_knots(offsets)[r] and point idx[r]."""
    return eval_pairs(blob, knots, points, row_knots(offsets), np.asarray(idx, np.int64))


def projection_matrix(i: int, N: int, n: int = N_CONF, state_dim: int | None = None):
    """P_i in R^{n x N*state_dim} (0-based knot i): I_n at the columns of q_i."""
    sd = 2 * n if state_dim is None else state_dim
    P = np.zeros((n, N * sd))
    P[np.arange(n), sd * i + np.arange(n)] = 1.0
    return P


def assemble_jacobian(grad_rows, offsets, n: int = N_CONF, state_dim: int | None = None):
    """Dense (sum m_i) x N*state_dim Jacobian: block i = grad_rows[block i] @ P_i."""
    off = np.asarray(offsets, np.int64)
    N = len(off) - 1
    g = np.asarray(grad_rows, np.float64).reshape(-1, n)
    blocks = [g[off[i]:off[i + 1]] @ projection_matrix(i, N, n, state_dim) for i in range(N)]
    sd = 2 * n if state_dim is None else state_dim
    return np.concatenate(blocks, axis=0) if blocks else np.zeros((0, N * sd))


def stacked_constraints_of_state(blob: bytes, X, points, offsets, idx, n: int = N_CONF):
    """c_gcdf as a function of the full decision vector X = [x_1, ..., x_N],
    x_i = [q_i, v_i] in R^{2n} (float64 throughout); used for finite differences."""
    off = np.asarray(offsets, np.int64)
    N = len(off) - 1
    q = np.asarray(X, np.float64).reshape(N, 2 * n)[:, :n]
    d, _ = eval_grad(blob, q, np.asarray(points, np.float64), with_grad=False)
    rows = row_knots(off)
    return d[rows, np.asarray(idx, np.int64)]
