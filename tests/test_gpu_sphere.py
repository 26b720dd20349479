"""Sphere obstacles (x, y, z, r) with the 10-input network [p', r, a] of the
primitive-aware extension (Sec. VII): HIP path vs the FP64 oracle and vs the
point path, through the C ABI (needs an MI355X).

Tolerances as for point obstacles (the arithmetic differs only by one more
input-layer product per row): FP32 |dd| <= 5e-5, relative J <= 5e-5; BF16X2
|dd| <= 1e-3, relative J <= 1e-2; BF16 about twice its measured maxima (0.07, 0.08).
"""
import time

import numpy as np
import pytest

from paper_2601_18548_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp32": (5e-5, 5e-5), "bf16x2": (1e-3, 1e-2), "bf16x2_f16": (1e-3, 1e-2), "bf16": (0.07, 0.08)}
GiB = 1 << 30


@pytest.fixture(scope="module")
def gcdf():
    import paper_2601_18548_amd as g

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    g.library()
    return g


def cu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rel_j_err(J, Jr):
    J = J.reshape(-1, 9).astype(np.float64)
    Jr = Jr.reshape(-1, 9)
    nr = np.linalg.norm(Jr, axis=1)
    return np.linalg.norm(J - Jr, axis=1) / np.maximum(nr, 1e-3 * np.median(nr))


@pytest.mark.parametrize("precision", ["fp32", "bf16x2", "bf16x2_f16", "bf16"])
@pytest.mark.parametrize("width", [256, 512])
def test_sphere_query_matches_oracle(gcdf, oracle_mod, precision, width):
    w = wl.weights(width, seed=41, in_dim=10)
    ctx = gcdf.Context(w.to_blob(), width, precision)
    assert ctx.obstacle_dim == 4
    for K, Np, seed in [(16, 64, 1), (3, 100, 7)]:
        print("case sphere width=%d precision=%s K=%d Np=%d" % (width, precision, K, Np), flush=True)
        k = wl.knots(K, seed)
        s = wl.spheres(Np, seed + 1)
        d, J = ctx.eval_grad(cu(k), cu(s))
        torch.cuda.synchronize()
        d, J = d.cpu().numpy(), J.cpu().numpy()
        dr, Jr = oracle_mod.eval_grad(w.to_blob(), k, s)
        dd, rj = np.abs(d - dr), rel_j_err(J, Jr)
        print("  |dd| max %.3e relJ max %.3e" % (dd.max(), rj.max()), flush=True)
        tol_d, tol_j = TOL[precision]
        assert np.all(np.isfinite(d)) and np.all(np.isfinite(J))
        assert dd.max() <= tol_d and rj.max() <= tol_j


@pytest.mark.parametrize("precision", ["fp32", "bf16x2", "bf16x2_f16"])
def test_zero_radius_column_equals_point_network_bitwise(gcdf, precision):
    """A sphere network whose radius column is zero and the point network
    without that column run the same arithmetic: equal bit for bit."""
    w10 = wl.weights(256, seed=42, in_dim=10)
    w10.mats[0][:, 3] = 0.0
    w9 = wl.Weights(256, 4, [np.delete(w10.mats[0], 3, axis=1)] + w10.mats[1:], list(w10.biases), 9)
    k = wl.knots(9, 2)
    s = wl.spheres(777, 3)
    c10 = gcdf.Context(w10.to_blob(), 256, precision)
    c9 = gcdf.Context(w9.to_blob(), 256, precision)
    d10, J10 = c10.eval_grad(cu(k), cu(s))
    d9, J9 = c9.eval_grad(cu(k), cu(s[:, :3]))
    torch.cuda.synchronize()
    assert torch.equal(d10, d9) and torch.equal(J10, J9)


def test_sphere_eval_knot_min_and_jmin_consistent(gcdf):
    w = wl.weights(512, seed=43, in_dim=10)
    ctx = gcdf.Context(w.to_blob(), 512, "bf16x2")
    k, s = cu(wl.knots(21, 4)), cu(wl.spheres(1500, 5))
    d, J = ctx.eval_grad(k, s)
    assert torch.equal(ctx.eval(k, s), d)
    dmin, am, Jm = ctx.knot_min(k, s, with_jacobian=True)
    torch.cuda.synchronize()
    dn, Jn = d.cpu().numpy(), J.cpu().numpy()
    am = am.cpu().numpy()
    assert np.array_equal(dmin.cpu().numpy(), dn.min(axis=1)) and np.array_equal(am, dn.argmin(axis=1))
    assert np.array_equal(Jm.cpu().numpy(), Jn[np.arange(21), am])


@pytest.mark.parametrize("precision", ["bf16x2", "fp32"])
def test_sphere_partitions_and_csr(gcdf, oracle_mod, precision):
    from oracle import constraints as cons

    w = wl.weights(256, seed=44, in_dim=10)
    ctx = gcdf.Context(w.to_blob(), 256, precision)
    N, M = 20, 5000
    k = wl.trajectory(N, 6)
    k[4, :2] += 50.0  # one empty partition
    s = wl.spheres(M, 7)
    kt, st = cu(k), cu(s)
    off, idx = ctx.partition(kt, st, 0.8, ref_stride=9)
    want_off, want_idx = cons.partition(k[:, :2], s, 0.8)
    assert np.array_equal(off.cpu().numpy(), want_off) and np.array_equal(idx.cpu().numpy(), want_idx)
    c, J = ctx.eval_grad_csr(kt, st, off, idx)
    d, Jd = ctx.eval_grad(kt, st)
    torch.cuda.synchronize()
    rows = cons.row_knots(want_off)
    ix = want_idx.astype(np.int64)
    cn, Jn = c.cpu().numpy(), J.cpu().numpy()
    assert np.array_equal(cn, d.cpu().numpy()[rows, ix]) and np.array_equal(Jn, Jd.cpu().numpy()[rows, ix])
    sel = np.random.default_rng(8).choice(len(ix), size=min(400, len(ix)), replace=False)
    dr, Jr = cons.constraints(w.to_blob(), k, s, want_off, ix)
    tol_d, tol_j = TOL[precision]
    assert np.abs(cn[sel] - dr[sel]).max() <= tol_d
    assert rel_j_err(Jn[sel], Jr[sel]).max() <= tol_j


def test_sphere_bad_index_gives_nan_row(gcdf):
    w = wl.weights(256, seed=45, in_dim=10)
    ctx = gcdf.Context(w.to_blob(), 256, "bf16x2")
    k, s = cu(wl.trajectory(2, 11)), cu(wl.spheres(50, 12))
    off = torch.tensor([0, 2, 4], dtype=torch.int64, device="cuda")
    idx = torch.tensor([0, 50, -3, 49], dtype=torch.int32, device="cuda")
    c, J = ctx.eval_grad_csr(k, s, off, idx)
    d, _ = ctx.eval_grad(k, s)
    cn, Jn, dn = c.cpu().numpy(), J.cpu().numpy(), d.cpu().numpy()
    assert np.isnan(cn[1]) and np.isnan(cn[2]) and np.all(np.isnan(Jn[[1, 2]]))
    assert cn[0] == dn[0, 0] and cn[3] == dn[1, 49]


@pytest.mark.parametrize("precision", ["bf16x2", "bf16x2_f16"])
def test_sphere_serving_matches_one_shot_bitwise(gcdf, precision):
    w = wl.weights(256, seed=46, in_dim=10)
    srv = gcdf.Context(w.to_blob(), 256, precision, serve_mem_budget=2 * GiB, serve_slots=8)
    one = gcdf.Context(w.to_blob(), 256, precision)
    reqs = []
    for i, (K, Np) in enumerate([(20, 1000), (7, 333), (40, 2100)]):
        k, s = cu(wl.knots(K, 60 + i)), cu(wl.spheres(Np, 70 + i))
        out = (torch.full((K, Np), float("nan"), device="cuda"), torch.full((K, Np, 9), float("nan"), device="cuda"),
               torch.full((K,), float("nan"), device="cuda"), torch.full((K,), -7, dtype=torch.int32, device="cuda"))
        reqs.append((k, s, out, srv.submit(k, s, *out)))
    t0 = time.time()
    for _, _, _, t in reqs:
        while not srv.poll(t):
            assert time.time() - t0 < 60, "serving did not finish"
            time.sleep(0.0005)
    for k, s, (d, J, dm, am), _ in reqs:
        dr, Jr = one.eval_grad(k, s)
        dmr, amr = one.knot_min(k, s)
        torch.cuda.synchronize()
        assert torch.equal(d, dr) and torch.equal(J, Jr) and torch.equal(dm, dmr) and torch.equal(am, amr)
    with pytest.raises(ValueError):
        srv.submit(reqs[0][0], reqs[0][1][:, :3].contiguous(), reqs[0][2][0])
    srv.close()


def test_point_shaped_input_is_rejected(gcdf):
    w = wl.weights(256, seed=47, in_dim=10)
    ctx = gcdf.Context(w.to_blob(), 256, "fp32")
    with pytest.raises(ValueError):
        ctx.eval(cu(wl.knots(2, 1)), cu(wl.points_uniform(5, 2)))
    bad = bytearray(w.to_blob())
    bad[8:12] = (11).to_bytes(4, "little")
    with pytest.raises(gcdf.GcdfError):
        gcdf.Context(bytes(bad), 256, "fp32")


def test_sphere_workload_full_size_sampled(gcdf, oracle_mod):
    """The benchmark's sphere workload (128 knots x 16,384 spheres, width 512,
    BF16X2) at full size, checked on sampled pairs and the per-knot minimum."""
    wk = wl.workload("sphere")
    print("full-size workload sphere: K=%d Np=%d width=%d %s" % (wk.K, wk.Np, wk.width, wk.precision), flush=True)
    ctx = gcdf.Context(wk.weights.to_blob(), wk.width, wk.precision)
    kt, st = cu(wk.knots), cu(wk.points)
    d, J = ctx.eval_grad(kt, st)
    torch.cuda.synchronize()
    d, J = d.cpu().numpy(), J.cpu().numpy()
    r = np.random.default_rng(0)
    ki, pi = r.integers(0, wk.K, 1500), r.integers(0, wk.Np, 1500)
    ki[:3] = [0, wk.K - 1, wk.K // 2]
    pi[:3] = [0, wk.Np - 1, wk.Np - 1]
    dr, Jr = oracle_mod.eval_pairs(wk.weights.to_blob(), wk.knots, wk.points, ki, pi)
    dd, rj = np.abs(d[ki, pi] - dr), rel_j_err(J[ki, pi], Jr)
    print("  sampled |dd| max %.3e relJ max %.3e" % (dd.max(), rj.max()), flush=True)
    assert np.all(np.isfinite(d)) and np.all(np.isfinite(J))
    assert dd.max() <= 1e-3 and rj.max() <= 1e-2
    dmin, am = ctx.knot_min(kt, st)
    dmin, am = dmin.cpu().numpy(), am.cpu().numpy()
    assert np.array_equal(dmin, d.min(axis=1)) and np.array_equal(am, d.argmin(axis=1))
