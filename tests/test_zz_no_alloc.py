"""gcdf_query_noalloc (the entry point that allocates nothing) against gcdf_query,
through the C ABI: the same kernels, so every output must be bitwise equal.

Two calls in a row share the GPU's fixed key array; the second, smaller call uses
other knots, so keys left over from the first would corrupt its minima unless
the call clears them.  Calls beyond the array's 65,536 knots are rejected.
"""
import ctypes

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


def _outputs(K, Np):
    z = dict(device="cuda")
    return (torch.full((K, Np), float("nan"), **z), torch.full((K, Np, 9), float("nan"), **z),
            torch.full((K,), float("nan"), **z), torch.full((K,), -5, dtype=torch.int32, **z),
            torch.full((K, 9), float("nan"), **z))


def _call(g, fn, ctx, kt, pt, outs):
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = [ctypes.c_void_p(t.data_ptr()) for t in outs]
    st = fn(ctx._h, ctypes.c_void_p(kt.data_ptr()), kt.shape[0], ctypes.c_void_p(pt.data_ptr()), pt.shape[0],
            *p, s)
    return st


@pytest.mark.parametrize("precision,width", [("bf16x2_f16", 256), ("fp32", 256), ("bf16x2", 512)])
def test_noalloc_matches_query_on_two_calls(gcdf, precision, width):
    lib = gcdf.library()
    w = wl.weights(width, seed=71)
    ctx = gcdf.Context(w.to_blob(), width, precision)
    for K, Np, seed in [(300, 1000, 5), (37, 555, 9)]:  # the second call smaller, other knots
        print("case noalloc %s w%d K=%d Np=%d" % (precision, width, K, Np), flush=True)
        kt = torch.from_numpy(wl.knots(K, seed)).cuda()
        pt = torch.from_numpy(wl.points_patches(Np, seed + 1)).cuda()
        a = _outputs(K, Np)
        b = _outputs(K, Np)
        assert _call(gcdf, lib.gcdf_query_noalloc, ctx, kt, pt, a) == gcdf.OK
        torch.cuda.synchronize()
        assert _call(gcdf, lib.gcdf_query, ctx, kt, pt, b) == gcdf.OK
        torch.cuda.synchronize()
        for x, y in zip(a, b):
            assert torch.equal(x, y)
        d = b[0]
        assert torch.equal(a[2], d.min(dim=1).values)
        assert torch.equal(a[3].long(), d.argmin(dim=1))
    ctx.close()


def test_noalloc_limits_and_outputs_subsets(gcdf):
    lib = gcdf.library()
    w = wl.weights(256, seed=72)
    ctx = gcdf.Context(w.to_blob(), 256, "bf16x2_f16")
    K = 65537
    kt = torch.from_numpy(wl.knots(K, 3)).cuda()
    pt = torch.from_numpy(wl.points_uniform(1, 4)).cuda()
    dmin = torch.empty(K, device="cuda")
    am = torch.empty(K, dtype=torch.int32, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = lib.gcdf_query_noalloc(ctx._h, kt.data_ptr(), K, pt.data_ptr(), 1, None, None, dmin.data_ptr(),
                                am.data_ptr(), None, s)
    assert st == gcdf.EINVAL and b"no-allocation" in lib.gcdf_last_error(None)
    # without the minimum the key array is not used: any K
    d = torch.empty((K, 1), device="cuda")
    assert lib.gcdf_query_noalloc(ctx._h, kt.data_ptr(), K, pt.data_ptr(), 1, d.data_ptr(), None, None, None,
                                  None, s) == gcdf.OK
    d2 = ctx.eval(kt, pt)
    torch.cuda.synchronize()
    assert torch.equal(d, d2)
    # the binding's flag routes through the same entry point
    kk, pp = kt[:40].contiguous(), torch.from_numpy(wl.points_patches(300, 5)).cuda()
    dm1, am1 = torch.empty(40, device="cuda"), torch.empty(40, dtype=torch.int32, device="cuda")
    ctx.query(kk, pp, dmin=dm1, argmin=am1, noalloc=True)
    dm2, am2 = ctx.knot_min(kk, pp)
    torch.cuda.synchronize()
    assert torch.equal(dm1, dm2) and torch.equal(am1, am2)
    ctx.close()
