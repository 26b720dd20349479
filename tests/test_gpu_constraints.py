"""Obstacle partitions, the CSR query and the sparse constraint Jacobian on the
GPU (Sec. IV-A), through the C ABI, against the oracle.

Partitions and the sparsity pattern are integer work: bit-exact.  The CSR
query runs the same per-pair code as the dense query, so its rows are bitwise
equal to the dense entries of the same pairs; against the FP64 oracle it has
the dense query's tolerance (|dd| <= 1e-3, relative J error <= 1e-2 with hi/lo
BF16; 5e-5 with FP32).
"""
import numpy as np
import pytest

from paper_2601_18548_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gcdf():
    import paper_2601_18548_amd as g

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    g.library()
    return g


@pytest.fixture(scope="module")
def cons(oracle_mod):
    from oracle import constraints

    return constraints


@pytest.fixture(scope="module")
def weights():
    return wl.weights(256, seed=61)


def cu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("N,M,radius,seed", [(7, 1000, 1.2, 1), (33, 10000, 0.9, 2), (128, 16384, 1.5, 3)])
def test_partitions_bit_exact(gcdf, cons, weights, N, M, radius, seed):
    k = wl.trajectory(N, seed)
    p = wl.points_patches(M, seed + 10)
    ctx = gcdf.Context(weights.to_blob(), 256, "bf16x2")
    off, idx = ctx.partition(cu(k), cu(p), radius, ref_stride=9)
    want_off, want_idx = cons.partition(k[:, :2], p, radius)
    assert np.array_equal(off.cpu().numpy(), want_off)
    assert np.array_equal(idx.cpu().numpy(), want_idx)
    # the same from a separate (N, 2) array of base positions
    off2, idx2 = ctx.partition(cu(k[:, :2].copy()), cu(p), radius)
    assert torch.equal(off, off2) and torch.equal(idx, idx2)


def test_partitions_with_empty_rows_and_capacity(gcdf, cons, weights):
    k = wl.trajectory(12, 4)
    k[3:6, :2] += 50.0  # far from every point: empty partitions in the middle
    k[0, :2] += 50.0    # and the first
    p = wl.points_patches(3000, 5)
    ctx = gcdf.Context(weights.to_blob(), 256, "bf16x2")
    off, idx = ctx.partition(cu(k), cu(p), 1.0, ref_stride=9)
    want_off, want_idx = cons.partition(k[:, :2], p, 1.0)
    assert np.array_equal(off.cpu().numpy(), want_off) and np.array_equal(idx.cpu().numpy(), want_idx)
    assert (np.diff(want_off) == 0).sum() == 4
    # capacity below the total: only the first `capacity` entries are written
    total = int(want_off[-1])
    cap = total // 2
    buf = torch.full((total,), -5, dtype=torch.int32, device="cuda")
    lib = gcdf.library()
    st = lib.gcdf_partition_fill(ctx._h, cu(k).data_ptr(), 12, 9, cu(p).data_ptr(), 3000, 1.0, off.data_ptr(),
                                 buf.data_ptr(), cap, None)
    torch.cuda.synchronize()
    assert st == gcdf.OK
    b = buf.cpu().numpy()
    assert np.array_equal(b[:cap], want_idx[:cap]) and np.all(b[cap:] == -5)


@pytest.mark.parametrize("precision,tol_d,tol_j", [("bf16x2", 1e-3, 1e-2), ("bf16x2_f16", 1e-3, 1e-2), ("fp32", 5e-5, 5e-5)])
def test_csr_query_matches_dense_and_oracle(gcdf, cons, weights, precision, tol_d, tol_j):
    N, M = 24, 4000
    k = wl.trajectory(N, 6)
    k[5, :2] += 50.0  # one empty partition
    p = wl.points_patches(M, 7)
    ctx = gcdf.Context(weights.to_blob(), 256, precision)
    kt, pt = cu(k), cu(p)
    off, idx = ctx.partition(kt, pt, 1.1, ref_stride=9)
    c, J = ctx.eval_grad_csr(kt, pt, off, idx)
    d, Jd = ctx.eval_grad(kt, pt)
    torch.cuda.synchronize()
    o, ix = off.cpu().numpy(), idx.cpu().numpy().astype(np.int64)
    rows = cons.row_knots(o)
    cn, Jn = c.cpu().numpy(), J.cpu().numpy()
    assert np.array_equal(cn, d.cpu().numpy()[rows, ix])
    assert np.array_equal(Jn, Jd.cpu().numpy()[rows, ix])
    # value-only form
    c2 = ctx.eval_grad_csr(kt, pt, off, idx, with_grad=False)
    assert torch.equal(c2, c)
    # oracle on a sample of rows
    sel = np.random.default_rng(8).choice(len(ix), size=min(600, len(ix)), replace=False)
    dr, Jr = cons.constraints(weights.to_blob(), k, p, o, ix)
    assert np.abs(cn[sel] - dr[sel]).max() <= tol_d
    nr = np.linalg.norm(Jr[sel], axis=1)
    rel = np.linalg.norm(Jn[sel] - Jr[sel], axis=1) / np.maximum(nr, 1e-3 * np.median(nr))
    assert rel.max() <= tol_j


def test_csr_query_many_knots_matches_dense(gcdf, cons, weights):
    """2,500 knots (more than one knot per thread of the tile-offset scan, the last
    segments ragged), partitions of every size including empty ones: every CSR row
    bitwise equal to the dense query's value at that (knot, point)."""
    N, M = 2500, 1500
    k = wl.trajectory(N, 31)
    k[7::97, :2] += 50.0  # empty partitions spread over the scan's segments
    p = wl.points_patches(M, 32)
    ctx = gcdf.Context(weights.to_blob(), 256, "bf16x2")
    kt, pt = cu(k), cu(p)
    off, idx = ctx.partition(kt, pt, 0.6, ref_stride=9)
    o = off.cpu().numpy()
    print("case CSR many knots: N=%d rows=%d empty=%d" % (N, int(o[-1]), int((np.diff(o) == 0).sum())), flush=True)
    assert (np.diff(o) == 0).sum() >= 20 and o[-1] > 0
    c = ctx.eval_grad_csr(kt, pt, off, idx, with_grad=False)
    d, _ = ctx.eval_grad(kt, pt)
    torch.cuda.synchronize()
    rows = cons.row_knots(o)
    assert np.array_equal(c.cpu().numpy(), d.cpu().numpy()[rows, idx.cpu().numpy().astype(np.int64)])
    ctx.close()


def test_jacobian_pattern_bit_exact(gcdf, cons, weights):
    N = 10
    k = wl.trajectory(N, 9)
    k[4, :2] += 50.0
    p = wl.points_patches(500, 10)
    ctx = gcdf.Context(weights.to_blob(), 256, "bf16x2")
    kt, pt = cu(k), cu(p)
    off, idx = ctx.partition(kt, pt, 1.0, ref_stride=9)
    total = idx.shape[0]
    c, J = ctx.eval_grad_csr(kt, pt, off, idx)
    row_ptr, cols = ctx.jacobian_pattern(off, total, state_dim=18)
    rp, cl, Jn = row_ptr.cpu().numpy(), cols.cpu().numpy(), J.cpu().numpy()
    assert np.array_equal(rp, 9 * np.arange(total + 1))
    dense = np.zeros((total, 18 * N))
    for r in range(total):
        dense[r, cl[rp[r]:rp[r + 1]]] = Jn[r]
    want = cons.assemble_jacobian(Jn.astype(np.float64), off.cpu().numpy())
    assert np.array_equal(dense, want)
    # a column offset and a wider state
    row_ptr, cols = ctx.jacobian_pattern(off, total, state_dim=25, col0=7)
    rows = cons.row_knots(off.cpu().numpy())
    want_cols = 7 + 25 * rows[:, None] + np.arange(9)[None, :]
    assert np.array_equal(cols.cpu().numpy().reshape(total, 9), want_cols)


def test_bad_point_index_gives_nan_row(gcdf, weights):
    k = wl.trajectory(3, 11)
    p = wl.points_patches(100, 12)
    ctx = gcdf.Context(weights.to_blob(), 256, "bf16x2")
    off = torch.tensor([0, 3, 3, 6], dtype=torch.int64, device="cuda")
    idx = torch.tensor([0, 100, 5, -1, 99, 7], dtype=torch.int32, device="cuda")
    c, J = ctx.eval_grad_csr(cu(k), cu(p), off, idx)
    d, Jd = ctx.eval_grad(cu(k), cu(p))
    cn, Jn = c.cpu().numpy(), J.cpu().numpy()
    assert np.isnan(cn[1]) and np.isnan(cn[3]) and np.all(np.isnan(Jn[[1, 3]]))
    dn = d.cpu().numpy()
    assert cn[0] == dn[0, 0] and cn[2] == dn[0, 5] and cn[4] == dn[2, 99] and cn[5] == dn[2, 7]


def test_argument_errors(gcdf, weights):
    ctx = gcdf.Context(weights.to_blob(), 256, "bf16x2")
    lib = gcdf.library()
    k, p = cu(wl.trajectory(4, 13)), cu(wl.points_patches(64, 14))
    off = torch.zeros(5, dtype=torch.int64, device="cuda")
    for stride, radius in ((1, 1.0), (9, -1.0), (9, float("nan")), (9, float("inf"))):
        st = lib.gcdf_partition_count(ctx._h, k.data_ptr(), 4, stride, p.data_ptr(), 64, radius, off.data_ptr(), None)
        assert st == gcdf.EINVAL
    assert lib.gcdf_partition_count(ctx._h, k.data_ptr(), 0, 9, p.data_ptr(), 64, 1.0, off.data_ptr(), None) == gcdf.EINVAL
    assert lib.gcdf_jacobian_pattern(ctx._h, off.data_ptr(), 4, 10, 8, 0, off.data_ptr(), off.data_ptr(), None) == gcdf.EINVAL
    c = torch.empty(1, device="cuda")
    # total == 0: nothing to do
    assert lib.gcdf_eval_grad_csr(ctx._h, k.data_ptr(), 4, p.data_ptr(), 64, None, None, 0, c.data_ptr(), None,
                                  None) == gcdf.OK
    assert lib.gcdf_eval_grad_csr(ctx._h, k.data_ptr(), 4, p.data_ptr(), 64, off.data_ptr(), None, 3, c.data_ptr(),
                                  None, None) == gcdf.EINVAL


M_DIAG = [2.0, 2.0, 0.5, 1.0, 1.5, 1.0, 1.0, 3.0, 1.0]


@pytest.mark.parametrize("precision", ["bf16x2", "fp32"])
def test_projection_matches_oracle(gcdf, oracle_mod, weights, precision):
    K, Np = 16, 700  # 11,200 rows: a ragged last block
    k, p = wl.knots(K, 20), wl.points_patches(Np, 21)
    ctx = gcdf.Context(weights.to_blob(), 256, precision)
    kt, pt = cu(k), cu(p)
    d, J = ctx.eval_grad(kt, pt)
    qz, eik = ctx.project(kt, d, J, M_DIAG)
    torch.cuda.synchronize()
    dn, Jn, qn, en = d.cpu().numpy(), J.cpu().numpy(), qz.cpu().numpy(), eik.cpu().numpy()
    # the kernel on its own inputs: the FP64 formula, float32 rounding only
    qr, er = oracle_mod.project(k[:, None, :], dn, Jn, M_DIAG)
    scale = 1.0 + np.abs(k[:, None, :]) + np.abs(dn[..., None] * Jn / np.asarray(M_DIAG))
    assert np.all(np.abs(qn - qr) <= 4e-7 * scale)
    assert np.all(np.abs(en - er) <= 4e-7 * er + 1e-30)
    # end to end against the oracle's distances and gradients, on a sample
    ki = np.arange(K).repeat(10)
    pi = np.random.default_rng(22).integers(0, Np, len(ki))
    d0, J0 = oracle_mod.eval_pairs(weights.to_blob(), k, p, ki, pi)
    q0, e0 = oracle_mod.project(k[ki], d0, J0, M_DIAG)
    tol_d, tol_j = (1e-3, 1e-2) if precision == "bf16x2" else (5e-5, 5e-5)
    # |dqz| <= |dd| |M^-1 J| + |d| max(M^-1) |dJ| and |deik| <= sqrt(max(M^-1)) |dJ|,
    # with |dd| <= tol_d and |dJ| <= tol_j max(|J|, 1e-3 median |J|) (the query's bar)
    minv = 1.0 / np.asarray(M_DIAG)
    nj = np.linalg.norm(J0, axis=1)
    dj = tol_j * np.maximum(nj, 1e-3 * np.median(nj))
    bound_q = tol_d * np.linalg.norm(minv * J0, axis=1) + np.abs(d0) * minv.max() * dj + 1e-5
    assert np.all(np.linalg.norm(qn[ki, pi] - q0, axis=1) <= bound_q)
    assert np.all(np.abs(en[ki, pi] - e0) <= np.sqrt(minv.max()) * dj + 1e-6)
    # single outputs give the same values
    q_only, _ = ctx.project(kt, d, J, M_DIAG, with_eik=False)
    _, e_only = ctx.project(kt, d, J, M_DIAG, with_qz=False)
    assert torch.equal(q_only, qz) and torch.equal(e_only, eik)


def test_projection_csr_equals_dense(gcdf, cons, weights):
    k = wl.trajectory(20, 23)
    k[7, :2] += 50.0
    p = wl.points_patches(2500, 24)
    ctx = gcdf.Context(weights.to_blob(), 256, "bf16x2")
    kt, pt = cu(k), cu(p)
    off, idx = ctx.partition(kt, pt, 1.2, ref_stride=9)
    c, J = ctx.eval_grad_csr(kt, pt, off, idx)
    qz, eik = ctx.project(kt, c, J, M_DIAG, offsets=off)
    d, Jd = ctx.eval_grad(kt, pt)
    qd, ed = ctx.project(kt, d, Jd, M_DIAG)
    torch.cuda.synchronize()
    rows = cons.row_knots(off.cpu().numpy())
    ix = idx.cpu().numpy().astype(np.int64)
    assert np.array_equal(qz.cpu().numpy(), qd.cpu().numpy()[rows, ix])
    assert np.array_equal(eik.cpu().numpy(), ed.cpu().numpy()[rows, ix])


def test_projection_argument_errors(gcdf, weights):
    ctx = gcdf.Context(weights.to_blob(), 256, "bf16x2")
    lib = gcdf.library()
    import ctypes

    k = cu(wl.knots(2, 25))
    d = torch.zeros((2, 3), device="cuda")
    J = torch.zeros((2, 3, 9), device="cuda")
    out = torch.empty((2, 3, 9), device="cuda")
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        m = (ctypes.c_float * 9)(*([1.0] * 8 + [bad]))
        assert lib.gcdf_project(ctx._h, k.data_ptr(), 2, 3, d.data_ptr(), J.data_ptr(), m, out.data_ptr(), None,
                                None) == gcdf.EINVAL
    m = (ctypes.c_float * 9)(*([1.0] * 9))
    assert lib.gcdf_project(ctx._h, k.data_ptr(), 2, 3, d.data_ptr(), J.data_ptr(), m, None, None, None) == gcdf.EINVAL
    assert lib.gcdf_project(ctx._h, k.data_ptr(), 0, 3, d.data_ptr(), J.data_ptr(), m, out.data_ptr(), None,
                            None) == gcdf.EINVAL
