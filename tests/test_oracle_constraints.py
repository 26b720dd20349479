"""Pins of the oracle's obstacle partitions and sparse constraint Jacobian
(Sec. IV-A): a k-d tree ball query (scipy) for the partitions, and central
finite differences of the stacked constraint vector with respect to the full
decision vector X = [x_1, ..., x_N], x_i = [q_i, v_i], for the Jacobian."""
import numpy as np
import pytest

from paper_2601_18548_amd import workloads as wl

scipy_spatial = pytest.importorskip("scipy.spatial")


@pytest.fixture(scope="module")
def cons(oracle_mod):
    from oracle import constraints

    return constraints


def _refs_and_points(N, M, seed):
    k = wl.knots(N, seed)
    p = wl.points_patches(M, seed + 1)
    return k, p


def test_partition_matches_kdtree_ball_query(cons):
    k, p = _refs_and_points(24, 3000, 7)
    radius = 1.3
    ref = k[:, :2]
    # drop points within 1e-4 of any partition boundary: there float32 and the
    # tree's float64 may legitimately decide differently
    dist = np.sqrt(((p[None, :, :2].astype(np.float64) - ref[:, None, :].astype(np.float64)) ** 2).sum(-1))
    keep = np.all(np.abs(dist - radius) > 1e-4, axis=0)
    p = p[keep]
    off, idx = cons.partition(ref, p, radius)
    assert off.dtype == np.int64 and idx.dtype == np.int32 and off[0] == 0 and off[-1] == len(idx)
    tree = scipy_spatial.cKDTree(p[:, :2].astype(np.float64))
    for i in range(len(ref)):
        want = np.sort(np.asarray(tree.query_ball_point(ref[i].astype(np.float64), radius), np.int64))
        got = idx[off[i]:off[i + 1]]
        assert np.all(np.diff(got) > 0)  # ascending, no repeats
        assert np.array_equal(got, want), i
    # the partitions overlap (neighbouring reference positions share points)
    assert len(idx) > len(np.unique(idx))


def test_partition_extremes(cons):
    k, p = _refs_and_points(5, 200, 8)
    off, idx = cons.partition(k[:, :2], p, 1e3)  # everything in every partition
    assert np.array_equal(off, np.arange(6) * 200)
    assert np.array_equal(idx, np.tile(np.arange(200, dtype=np.int32), 5))
    off, idx = cons.partition(k[:, :2] + 100.0, p, 1.0)  # nothing anywhere
    assert np.array_equal(off, np.zeros(6, np.int64)) and len(idx) == 0
    # a point exactly on the boundary belongs to the partition (<=)
    ref = np.array([[0.0, 0.0]], np.float32)
    pts = np.array([[0.5, 0.0, 0.3], [0.5000001, 0.0, 0.3]], np.float32)
    off, idx = cons.partition(ref, pts, 0.5)
    assert list(idx) == [0]


def test_projection_matrices(cons):
    N, n = 4, 9
    Ps = [cons.projection_matrix(i, N) for i in range(N)]
    for i in range(N):
        assert Ps[i].shape == (n, 2 * n * N)
        assert np.array_equal(Ps[i] @ Ps[i].T, np.eye(n))
        for j in range(N):
            if j != i:
                assert not np.any(Ps[i] @ Ps[j].T)
    # only configuration columns are hit, velocity columns never
    hit = sum(P.sum(0) for P in Ps)
    assert np.array_equal(hit, np.tile(np.r_[np.ones(n), np.zeros(n)], N))


def test_assembled_jacobian_matches_finite_differences_over_the_state(cons, oracle_mod):
    w = wl.weights(256, seed=41)
    blob = w.to_blob()
    N, n = 4, 9
    k, p = _refs_and_points(N, 60, 9)
    off, idx = cons.partition(k[:, :2], p, 1.6)
    assert 0 < len(idx) and np.all(np.diff(off) > 0)
    X = np.zeros((N, 2 * n))
    X[:, :n] = k
    X[:, n:] = np.random.default_rng(3).normal(size=(N, n))  # velocities: no effect on c
    X = X.ravel()
    _, J = oracle_mod.eval_grad(blob, k.astype(np.float64), p.astype(np.float64))
    rows = cons.row_knots(off)
    A = cons.assemble_jacobian(J[rows, idx.astype(np.int64)], off)
    assert A.shape == (len(idx), 2 * n * N)
    fd = np.zeros_like(A)
    for c in range(len(X)):
        h = 1e-6 * max(1.0, abs(X[c]))
        Xp, Xm = X.copy(), X.copy()
        Xp[c] += h
        Xm[c] -= h
        fd[:, c] = (cons.stacked_constraints_of_state(blob, Xp, p, off, idx)
                    - cons.stacked_constraints_of_state(blob, Xm, p, off, idx)) / (2 * h)
    assert np.abs(A - fd).max() <= 1e-6 * max(1.0, np.abs(A).max())
    # row r has exactly n structural non-zeros, at the columns of its own knot
    for r in range(len(idx)):
        nz = np.nonzero(A[r])[0]
        assert np.all((nz >= 2 * n * rows[r]) & (nz < 2 * n * rows[r] + n))


def test_constraint_vector_is_knot_major(cons, oracle_mod):
    w = wl.weights(256, seed=42)
    k, p = _refs_and_points(3, 50, 10)
    off, idx = cons.partition(k[:, :2], p, 1.5)
    c, G = cons.constraints(w.to_blob(), k, p, off, idx)
    d, J = oracle_mod.eval_grad(w.to_blob(), k, p)
    for i in range(3):
        sl = slice(off[i], off[i + 1])
        assert np.array_equal(c[sl], d[i, idx[sl]])
        assert np.array_equal(G[sl], J[i, idx[sl]])


def test_projection_closed_form_weighted_plane(oracle_mod):
    """Weighted distance to a hyperplane a.q = b: f = (a.q - b) / |a|_{M^-1}
    (the M-norm distance), grad f = a / |a|_{M^-1}; one projection step lands
    on the plane and the weighted eikonal norm is 1, for any diagonal M > 0."""
    r = np.random.default_rng(4)
    for _ in range(20):
        a = r.normal(size=9)
        b = r.normal()
        m = r.uniform(0.2, 20.0, size=9)
        q = r.normal(size=(5, 9))
        na = np.sqrt(np.sum(a * a / m))
        f = (q @ a - b) / na
        J = np.tile(a / na, (5, 1))
        qz, eik = oracle_mod.project(q, f, J, m)
        np.testing.assert_allclose(qz @ a, b, atol=1e-12)
        np.testing.assert_allclose(eik, 1.0, atol=1e-12)
        # q_z is the M-closest point of the plane: |q - q_z|_M = |f|
        np.testing.assert_allclose(np.sqrt(np.sum(m * (q - qz) ** 2, axis=1)), np.abs(f), rtol=1e-12)
