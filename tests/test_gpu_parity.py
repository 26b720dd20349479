"""HIP path vs the FP64 oracle, through the C ABI (needs an MI355X).

Tolerances (derivations in the design notes):
  FP32    : |dd| <= 5e-5 and per-pair relative J error <= 5e-5
  BF16X2  : |dd| <= 1e-3 and relative J error <= 1e-2 (the accuracy bar of the
            precision form), with the measured error printed
  BF16X2_F16 : the same bar (forward as BF16X2, reverse sweep in FP16: rounding
            emulation predicts relative J errors of a few 1e-3)
  BF16    : the fast mode does not meet that bar; it is checked against about
            twice its measured maxima (|dd| 3.4e-2, relative J 3.9e-2 over these
            cases): |dd| <= 0.07, relative J <= 0.08.
Relative J error per pair is |J - J_ref| / max(|J_ref|, 1e-3 * median |J_ref|).
"""
import numpy as np
import pytest

from paper_2601_18548_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp32": (5e-5, 5e-5), "bf16x2": (1e-3, 1e-2), "bf16x2_f16": (1e-3, 1e-2), "bf16": (0.07, 0.08)}


@pytest.fixture(scope="module")
def gcdf():
    import paper_2601_18548_amd as g

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    g.library()
    return g


def rel_j_err(J, Jr):
    J = J.reshape(-1, 9).astype(np.float64)
    Jr = Jr.reshape(-1, 9)
    nr = np.linalg.norm(Jr, axis=1)
    den = np.maximum(nr, 1e-3 * np.median(nr))
    return np.linalg.norm(J - Jr, axis=1) / den


def run_eval_grad(g, w, precision, k, p):
    ctx = g.Context(w.to_blob(), w.width, precision)
    kt = torch.from_numpy(k).cuda()
    pt = torch.from_numpy(p).cuda()
    d, J = ctx.eval_grad(kt, pt)
    torch.cuda.synchronize()
    return ctx, kt, pt, d.cpu().numpy(), J.cpu().numpy()


def report(name, dd, rj):
    print("%s: |dd| max %.3e mean %.3e | relJ max %.3e p99 %.3e mean %.3e" %
          (name, dd.max(), dd.mean(), rj.max(), np.percentile(rj, 99), rj.mean()), flush=True)


@pytest.mark.parametrize("precision", ["fp32", "bf16x2", "bf16x2_f16", "bf16"])
@pytest.mark.parametrize("width", [256, 512])
def test_small_workload_matches_oracle(gcdf, oracle_mod, precision, width):
    """16 knots x 64 points (the small workload's sizes) plus a ragged 3 x 100 case."""
    w = wl.weights(width, seed=3)
    for K, Np, seed in [(16, 64, 1), (3, 100, 7)]:
        k = wl.knots(K, seed)
        p = wl.points_uniform(Np, seed + 1)
        print("case width=%d precision=%s K=%d Np=%d" % (width, precision, K, Np), flush=True)
        _, _, _, d, J = run_eval_grad(gcdf, w, precision, k, p)
        dr, Jr = oracle_mod.eval_grad(w.to_blob(), k, p)
        dd = np.abs(d - dr)
        rj = rel_j_err(J, Jr)
        report("w%d %s K%d Np%d" % (width, precision, K, Np), dd, rj)
        tol_d, tol_j = TOL[precision]
        assert np.all(np.isfinite(d)) and np.all(np.isfinite(J))
        assert dd.max() <= tol_d
        assert rj.max() <= tol_j


def test_eval_and_knot_min_are_consistent_bitwise(gcdf):
    """d from eval == d from eval_grad; knot_min == min over that d (lowest index);
    Jmin == J at the argmin (the pair-list path runs the same arithmetic)."""
    w = wl.weights(256, seed=5)
    k = wl.knots(37, 2)
    p = wl.points_patches(1000, 3)
    for precision in ["fp32", "bf16x2"]:
        ctx, kt, pt, d, J = run_eval_grad(gcdf, w, precision, k, p)
        d2 = ctx.eval(kt, pt).cpu().numpy()
        assert np.array_equal(d, d2)
        dmin, am, Jm = ctx.knot_min(kt, pt, with_jacobian=True)
        torch.cuda.synchronize()
        dmin, am, Jm = dmin.cpu().numpy(), am.cpu().numpy(), Jm.cpu().numpy()
        assert np.array_equal(dmin, d.min(axis=1))
        assert np.array_equal(am, d.argmin(axis=1))
        assert np.array_equal(Jm, J[np.arange(len(k)), am])


def test_ties_pick_lowest_index(gcdf):
    """Duplicated points give exactly equal distances: the lowest index must win."""
    w = wl.weights(256, seed=6)
    k = wl.knots(5, 4)
    base = wl.points_uniform(70, 5)
    p = np.concatenate([base, base, base], 0)  # every distance appears 3 times
    ctx = gcdf.Context(w.to_blob(), 256, "bf16x2")
    kt, pt = torch.from_numpy(k).cuda(), torch.from_numpy(p).cuda()
    d = ctx.eval(kt, pt).cpu().numpy()
    dmin, am = ctx.knot_min(kt, pt)
    am = am.cpu().numpy()
    assert np.array_equal(am, d.argmin(axis=1))
    assert np.all(am < 70)


def test_single_pair_and_empty_tail(gcdf, oracle_mod):
    w = wl.weights(512, seed=8)
    k = wl.knots(1, 9)
    p = wl.points_uniform(1, 10)
    _, _, _, d, J = run_eval_grad(gcdf, w, "bf16x2", k, p)
    dr, Jr = oracle_mod.eval_grad(w.to_blob(), k, p)
    assert abs(d[0, 0] - dr[0, 0]) <= 1e-3
    assert rel_j_err(J, Jr).max() <= 1e-2


def test_argument_errors_do_not_launch(gcdf):
    w = wl.weights(256, seed=1)
    ctx = gcdf.Context(w.to_blob(), 256, "fp32")
    lib = gcdf.library()
    kt = torch.zeros((4, 9), device="cuda")
    pt = torch.zeros((4, 3), device="cuda")
    d = torch.zeros((4, 4), device="cuda")
    import ctypes
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.gcdf_eval(ctx._h, kt.data_ptr(), 0, pt.data_ptr(), 4, d.data_ptr(), s) == gcdf.EINVAL
    assert lib.gcdf_eval(ctx._h, None, 4, pt.data_ptr(), 4, d.data_ptr(), s) == gcdf.EINVAL
    assert lib.gcdf_eval(ctx._h, kt.data_ptr(), 4, pt.data_ptr(), -1, d.data_ptr(), s) == gcdf.EINVAL
    assert lib.gcdf_eval(ctx._h, kt.data_ptr(), 2**62, pt.data_ptr(), 2**10, d.data_ptr(), s) == gcdf.EINVAL
    assert b"overflow" in lib.gcdf_last_error(None)
    small = gcdf.Context(w.to_blob(), 256, "fp32", max_knots=2)
    with pytest.raises(gcdf.GcdfError):
        small.knot_min(kt, pt)


def _full_size_sampled(gcdf, oracle_mod, name, n_sample, precision=None):
    wk = wl.workload(name)
    if precision is not None:
        wk.precision = precision
    print("full-size workload %s: K=%d Np=%d width=%d %s" % (name, wk.K, wk.Np, wk.width, wk.precision), flush=True)
    ctx, kt, pt, d, J = run_eval_grad(gcdf, wk.weights, wk.precision, wk.knots, wk.points)
    r = np.random.default_rng(0)
    ki = r.integers(0, wk.K, n_sample)
    pi = r.integers(0, wk.Np, n_sample)
    # always include the first and last pair and the ragged end of a row
    ki[:3] = [0, wk.K - 1, wk.K // 2]
    pi[:3] = [0, wk.Np - 1, wk.Np - 1]
    dr, Jr = oracle_mod.eval_pairs(wk.weights.to_blob(), wk.knots, wk.points, ki, pi)
    dd = np.abs(d[ki, pi] - dr)
    rj = rel_j_err(J[ki, pi], Jr)
    report(name + " sampled", dd, rj)
    tol_d, tol_j = TOL[wk.precision]
    assert np.all(np.isfinite(d)) and np.all(np.isfinite(J))
    assert dd.max() <= tol_d and rj.max() <= tol_j
    # per-knot minimum: bitwise against the GPU's own d, value against the oracle
    dmin, am = ctx.knot_min(kt, pt)
    dmin, am = dmin.cpu().numpy(), am.cpu().numpy()
    assert np.array_equal(dmin, d.min(axis=1)) and np.array_equal(am, d.argmin(axis=1))
    dm_r, _ = oracle_mod.eval_pairs(wk.weights.to_blob(), wk.knots, wk.points, np.arange(wk.K), am)
    assert np.abs(dmin - dm_r).max() <= tol_d
    return d, J


def test_fp32_workload_full_size_sampled(gcdf, oracle_mod):
    _full_size_sampled(gcdf, oracle_mod, "fp32", 3000)


def test_bf16_workload_full_size_sampled_bf16x2(gcdf, oracle_mod):
    _full_size_sampled(gcdf, oracle_mod, "bf16", 1500, precision="bf16x2")


def test_bf16x2_f16_workload_full_size_sampled(gcdf, oracle_mod):
    """The 128 x 16,384 W=512 workload in the FP16-reverse mode, in the launch
    configuration the benchmark times; its d must equal BF16X2's bit for bit (the
    forward arithmetic is the same), its J within the bar."""
    d, J = _full_size_sampled(gcdf, oracle_mod, "bf16", 1500, precision="bf16x2_f16")
    wk = wl.workload("bf16")
    _, _, _, d2, J2 = run_eval_grad(gcdf, wk.weights, "bf16x2", wk.knots, wk.points)
    assert np.array_equal(d, d2)
    rj = rel_j_err(J, J2)
    print("bf16x2_f16 vs bf16x2 J over all pairs: max %.3e p99 %.3e" % (rj.max(), np.percentile(rj, 99)), flush=True)
    assert rj.max() <= 1e-2


@pytest.mark.parametrize("width", [256, 512])
def test_fp16_reverse_mode_ragged_and_value_only(gcdf, oracle_mod, width):
    """Ragged tiles, a single pair, and eval (no reverse sweep) in BF16X2_F16:
    eval's d equals eval_grad's bit for bit."""
    w = wl.weights(width, seed=11)
    for K, Np, seed in [(1, 1, 3), (5, 65, 4), (2, 127, 5)]:
        k = wl.knots(K, seed)
        p = wl.points_patches(Np, seed + 1)
        print("case width=%d bf16x2_f16 K=%d Np=%d" % (width, K, Np), flush=True)
        ctx, kt, pt, d, J = run_eval_grad(gcdf, w, "bf16x2_f16", k, p)
        dr, Jr = oracle_mod.eval_grad(w.to_blob(), k, p)
        assert np.abs(d - dr).max() <= 1e-3 and rel_j_err(J, Jr).max() <= 1e-2
        assert np.array_equal(ctx.eval(kt, pt).cpu().numpy(), d)


def test_outputs_past_32_bit_offsets(gcdf, oracle_mod):
    """1,024 knots x 262,143 points (the last tile of every row ragged), width 256,
    the benchmark precision: J holds 2.4e9 floats (9.7 GB), so element offsets pass
    2^31 and byte offsets 2^32.  Sampled pairs, the whole tail of the last row and
    the per-knot minimum are checked; the samples are gathered on the device."""
    K, Np = 1024, 262143
    w = wl.weights(256, seed=13)
    k = wl.knots(K, 21)
    p = wl.points_patches(Np, 22)
    print("case 32-bit offsets: K=%d Np=%d (J %.1f GB)" % (K, Np, K * Np * 36 / 1e9), flush=True)
    ctx = gcdf.Context(w.to_blob(), 256, "bf16x2_f16")
    kt, pt = torch.from_numpy(k).cuda(), torch.from_numpy(p).cuda()
    d, J = ctx.eval_grad(kt, pt)
    r = np.random.default_rng(1)
    ki = np.concatenate([r.integers(0, K, 400), np.full(70, K - 1), [0, K // 2]])
    pi = np.concatenate([r.integers(0, Np, 400), np.arange(Np - 70, Np), [0, Np - 1]])
    kd, pd = torch.from_numpy(ki).cuda(), torch.from_numpy(pi).cuda()
    ds, Js = d[kd, pd].cpu().numpy(), J[kd, pd].cpu().numpy()
    dr, Jr = oracle_mod.eval_pairs(w.to_blob(), k, p, ki, pi)
    dd, rj = np.abs(ds - dr), rel_j_err(Js, Jr)
    report("32-bit offsets sampled", dd, rj)
    assert dd.max() <= 1e-3 and rj.max() <= 1e-2
    dmin, am = ctx.knot_min(kt, pt)
    assert torch.equal(dmin, d.min(dim=1).values)
    assert torch.equal(d[torch.arange(K, device="cuda"), am.long()], dmin)
    del J, d
    torch.cuda.empty_cache()


def test_fp16_reverse_sweep_with_large_back_propagated_values(gcdf, oracle_mod):
    """BF16X2_F16 scales the reverse sweep by 2^6 into FP16 (largest finite 65504):
    a network whose output weights are 100x larger back-propagates values up to ~35
    (~2,200 after scaling), which must stay finite with the relative J error of the
    unscaled network; d scales by 100, so its error bar does too."""
    w = wl.weights(512, seed=3)
    w.mats[4] = (w.mats[4] * 100.0).astype(np.float32)
    k = wl.knots(8, 31)
    p = wl.points_patches(700, 32)
    print("case large reverse values: width 512 bf16x2_f16 K=8 Np=700", flush=True)
    _, _, _, d, J = run_eval_grad(gcdf, w, "bf16x2_f16", k, p)
    dr, Jr = oracle_mod.eval_grad(w.to_blob(), k, p)
    assert np.all(np.isfinite(d)) and np.all(np.isfinite(J))
    dd, rj = np.abs(d - dr), rel_j_err(J, Jr)
    report("large reverse values", dd, rj)
    assert dd.max() <= 100 * 1e-3 and rj.max() <= 1e-2


def test_fp16_reverse_overflow_is_reported(gcdf):
    """Output weights 10,000x larger back-propagate values of ~3e3 (~2e5 after the
    2^6 scale, past FP16's 65,504): J overflows while d stays finite.  The next
    query call on the context reports GCDF_ERANGE once, without launching; the call
    after it runs normally.  The BF16X2 context of the same network never flags."""
    w = wl.weights(512, seed=3)
    w.mats[4] = (w.mats[4] * 1.0e4).astype(np.float32)
    k = wl.knots(4, 33)
    p = wl.points_patches(300, 34)
    kt, pt = torch.from_numpy(k).cuda(), torch.from_numpy(p).cuda()
    print("case FP16 overflow: width 512 bf16x2_f16 K=4 Np=300", flush=True)
    ctx = gcdf.Context(w.to_blob(), 512, "bf16x2_f16")
    d, J = ctx.eval_grad(kt, pt)
    torch.cuda.synchronize()
    assert torch.isfinite(d).all() and not torch.isfinite(J).all()
    with pytest.raises(gcdf.GcdfError) as e:
        ctx.eval(kt, pt)
    assert e.value.status == gcdf.ERANGE
    d2 = ctx.eval(kt, pt)  # the flag was cleared by the report
    torch.cuda.synchronize()
    assert torch.equal(d2, d)
    ref = gcdf.Context(w.to_blob(), 512, "bf16x2")
    _, J3 = ref.eval_grad(kt, pt)
    torch.cuda.synchronize()
    assert torch.isfinite(J3).all()
    ref.eval(kt, pt)
    torch.cuda.synchronize()
    ctx.close()
    ref.close()


@pytest.mark.parametrize("precision", ["bf16x2_f16", "bf16x2"])
def test_off_grid_hidden_weights_error_measured(gcdf, oracle_mod, precision):
    """A network whose hidden weights are FP32 values off the BF16 grid (as FP32
    master weights of a trainer are): the BF16 precisions multiply the BF16-rounded
    hidden matrices, so against the FP64 oracle of the FP32 network they carry the
    rounding of the weights (~2^-9 relative each).  Measured and printed at W=512 on
    the benchmark point distribution, bounded by 0.1 (value and relative J) so a gross
    error still fails; with weights on the grid the same cases are under the 1e-3 /
    1e-2 bar (test_small_workload_matches_oracle)."""
    w = wl.weights(512, seed=3, bf16_hidden=False)
    k = wl.knots(16, 41)
    p = wl.points_patches(400, 42)
    print("case off-grid weights: width 512 %s K=16 Np=400" % precision, flush=True)
    _, _, _, d, J = run_eval_grad(gcdf, w, precision, k, p)
    dr, Jr = oracle_mod.eval_grad(w.to_blob(), k, p)
    dd, rj = np.abs(d - dr), rel_j_err(J, Jr)
    report("off-grid weights w512 %s" % precision, dd, rj)
    assert np.all(np.isfinite(d)) and np.all(np.isfinite(J))
    assert dd.max() <= 0.1 and rj.max() <= 0.1
