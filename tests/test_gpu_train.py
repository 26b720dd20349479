"""Training form on the GPU: weight gradients vs the FP64 oracle, finite
differences of the GPU loss, determinism, autograd + Adam.

Tolerances: FP32 mode, per parameter array, |g - g_ref| / |g_ref| <= 1e-5
(FP32 accumulation over a few hundred samples); BF16 mode (activations and
gradients rounded to BF16 for the matrix cores) <= 2e-2, printed.
"""
import numpy as np
import pytest

from paper_2601_18548_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NAMES = ["W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4", "w_out", "b_out"]


@pytest.fixture(scope="module")
def tr_mod():
    import paper_2601_18548_amd as g
    from paper_2601_18548_amd import train

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    g.library()
    return train


def batch(B, seed):
    k, p, noise = wl.training_batch(B, seed)
    y = np.random.default_rng(seed + 5).normal(0, 1, B).astype(np.float32)
    return k, p, y


def gpu_grads(tr_mod, precision, w, k, p, y):
    trainer = tr_mod.Trainer(256, precision, max_batch=len(k))
    params = tr_mod.flat_params(w)
    kt, pt = torch.from_numpy(k).cuda(), torch.from_numpy(p).cuda()
    d = trainer.forward(params, kt, pt)
    gd = (2.0 * (d - torch.from_numpy(y).cuda()) / len(k)).contiguous()
    g = trainer.backward(params, kt, pt, gd)
    torch.cuda.synchronize()
    return trainer, params, kt, pt, d.cpu().numpy(), g.cpu().numpy()


def split(flat, w):
    out, off = [], 0
    for a in w.flat_params():
        out.append(flat[off:off + a.size].reshape(a.shape))
        off += a.size
    return out


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("bf16", 2e-2)])
def test_weight_gradients_match_oracle(tr_mod, oracle_mod, precision, tol):
    w = wl.weights(256, seed=31, bf16_hidden=False)  # FP32 master weights, off the BF16 grid
    k, p, y = batch(300, 3)  # ragged: not a multiple of 64
    _, _, _, _, d, g = gpu_grads(tr_mod, precision, w, k, p, y)
    loss_ref, gref = oracle_mod.mse_grad(w.to_blob(), k.astype(np.float64), p.astype(np.float64), y)
    for name, a, b in zip(NAMES, split(g, w), gref):
        err = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        print("%s %-5s rel err %.2e" % (precision, name, err), flush=True)
        assert np.all(np.isfinite(a))
        assert err <= tol, name


# A batch past the chunk sizes of the reductions: on 256 compute units, 20
# weight-gradient GEMM chunks of 320 samples (the last one 101), 13 row-reduction
# chunks of 512 (FP32; the last 37), 97 tiles whose per-workgroup sums (BF16) are
# added over 97 workgroups, and a ragged last tile of 37 samples.
MULTI_B = 6181


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("bf16", 2e-2)])
def test_weight_gradients_match_oracle_multi_chunk(tr_mod, oracle_mod, precision, tol):
    """The chunked sums (GEMM chunks added in order, row-reduction chunks added in
    order) against the oracle's straight sum over all 6,181 samples."""
    w = wl.weights(256, seed=38, bf16_hidden=False)
    k, p, y = batch(MULTI_B, 13)
    print("case multi-chunk B=%d %s" % (MULTI_B, precision), flush=True)
    _, _, _, _, d, g = gpu_grads(tr_mod, precision, w, k, p, y)
    loss_ref, gref = oracle_mod.mse_grad(w.to_blob(), k.astype(np.float64), p.astype(np.float64), y)
    for name, a, b in zip(NAMES, split(g, w), gref):
        err = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        print("%s B=%d %-5s rel err %.2e" % (precision, MULTI_B, name, err), flush=True)
        assert np.all(np.isfinite(a))
        assert err <= tol, name


def fused_grads(tr_mod, precision, w, k, p, y):
    trainer = tr_mod.Trainer(256, precision, max_batch=len(k))
    params = tr_mod.flat_params(w)
    kt, pt = torch.from_numpy(k).cuda(), torch.from_numpy(p).cuda()
    d = torch.empty(len(k), device="cuda")
    loss, g = trainer.mse(params, kt, pt, torch.from_numpy(y).cuda(), d=d)
    torch.cuda.synchronize()
    return trainer, params, kt, pt, float(loss.item()), d.cpu().numpy(), g.cpu().numpy()


@pytest.mark.parametrize("B", [300, MULTI_B])
@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("bf16", 2e-2)])
def test_fused_mse_matches_oracle(tr_mod, oracle_mod, precision, tol, B):
    """gcdf_train_mse: the loss, the distances and the weight gradient of one fused
    pass against the oracle's (d is finished inside each tile before its reverse
    sweep, which the seeds 2 (d_i - y_i) / B come from)."""
    w = wl.weights(256, seed=40, bf16_hidden=False)
    k, p, y = batch(B, 15)
    print("case fused MSE B=%d %s" % (B, precision), flush=True)
    _, _, _, _, loss, d, g = fused_grads(tr_mod, precision, w, k, p, y)
    loss_ref, gref = oracle_mod.mse_grad(w.to_blob(), k.astype(np.float64), p.astype(np.float64), y)
    if precision == "fp32":
        dref, _ = oracle_mod.eval_pairs(w.to_blob(), k, p, np.arange(B), np.arange(B), with_grad=False)
        assert np.abs(d - dref).max() <= 1e-5
    lerr = abs(loss - loss_ref) / loss_ref
    print("%s B=%d loss %.6f ref %.6f rel err %.2e" % (precision, B, loss, loss_ref, lerr), flush=True)
    assert lerr <= (1e-5 if precision == "fp32" else 2e-2)
    for name, a, b in zip(NAMES, split(g, w), gref):
        err = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        print("%s B=%d fused %-5s rel err %.2e" % (precision, B, name, err), flush=True)
        assert np.all(np.isfinite(a))
        assert err <= tol, name


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("bf16", 1e-2)])
def test_fused_mse_agrees_with_forward_then_backward(tr_mod, precision, tol):
    """The fused pass against the separate forward + backward with torch's MSE seeds:
    the same distances, the loss of those distances, nearly the same gradient (the
    seeds round differently)."""
    w = wl.weights(256, seed=41, bf16_hidden=False)
    k, p, y = batch(MULTI_B, 16)
    _, _, _, _, d0, g0 = gpu_grads(tr_mod, precision, w, k, p, y)
    trainer, _, _, _, loss, d, g = fused_grads(tr_mod, precision, w, k, p, y)
    assert np.abs(d - d0).max() <= 1e-6 * max(1.0, np.abs(d0).max())
    ref = float(np.mean((d0.astype(np.float64) - y) ** 2))
    assert abs(loss - ref) <= 1e-5 * ref
    err = np.linalg.norm(g - g0) / np.linalg.norm(g0)
    print("%s fused vs separate gradient rel diff %.2e" % (precision, err), flush=True)
    assert err <= tol
    trainer.close()


EDGE_B = [1, 63, 64, 65, 64 * 256 + 5]


@pytest.mark.parametrize("B", EDGE_B)
def test_fused_mse_edge_batches_match_oracle(tr_mod, oracle_mod, B):
    """One sample, a partial tile, exactly one tile, one tile plus one sample, and 257
    tiles (one more than a round of workgroups on 256 compute units, the last one
    ragged): in FP32 the loss and every parameter array against the oracle."""
    w = wl.weights(256, seed=43, bf16_hidden=False)
    k, p, y = batch(B, 18)
    print("case fused MSE edge B=%d fp32" % B, flush=True)
    _, _, _, _, loss, d, g = fused_grads(tr_mod, "fp32", w, k, p, y)
    loss_ref, gref = oracle_mod.mse_grad(w.to_blob(), k.astype(np.float64), p.astype(np.float64), y)
    assert abs(loss - loss_ref) <= 1e-5 * loss_ref
    for name, a, b in zip(NAMES, split(g, w), gref):
        err = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        assert np.all(np.isfinite(a)) and err <= 1e-5, (name, err)


@pytest.mark.parametrize("B", EDGE_B)
def test_fused_mse_edge_batches_bf16(tr_mod, B):
    """The same batches in BF16 against the separate BF16 forward + backward (the same
    arithmetic but for the seeds' rounding).  Against the FP64 oracle the BF16 error
    of d (~1e-2 with FP32 hidden weights off the BF16 grid) can dominate a small
    gradient such as db_out = 2 mean(d - y), so the oracle bar of the large batches
    does not apply at every size."""
    w = wl.weights(256, seed=43, bf16_hidden=False)
    k, p, y = batch(B, 18)
    print("case fused MSE edge B=%d bf16" % B, flush=True)
    _, _, _, _, d0, g0 = gpu_grads(tr_mod, "bf16", w, k, p, y)
    _, _, _, _, loss, d, g = fused_grads(tr_mod, "bf16", w, k, p, y)
    assert np.abs(d - d0).max() <= 1e-6 * max(1.0, np.abs(d0).max())
    ref = float(np.mean((d0.astype(np.float64) - y) ** 2))
    assert abs(loss - ref) <= 1e-5 * ref
    for name, a, b in zip(NAMES, split(g, w), split(g0, w)):
        err = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        assert np.all(np.isfinite(a)) and err <= 1e-2, (name, err)


def test_fused_mse_rejects_bad_arguments(tr_mod):
    import ctypes

    from paper_2601_18548_amd import EINVAL, library

    w = wl.weights(256, seed=44, bf16_hidden=False)
    k, p, y = batch(100, 19)
    trainer = tr_mod.Trainer(256, "bf16", max_batch=100)
    params = tr_mod.flat_params(w)
    kt, pt, yt = torch.from_numpy(k).cuda(), torch.from_numpy(p).cuda(), torch.from_numpy(y).cuda()
    loss = torch.empty(1, device="cuda")
    grad = torch.empty_like(params)
    lib = library()
    args = [trainer._h, params.data_ptr(), kt.data_ptr(), pt.data_ptr(), 100, yt.data_ptr(), loss.data_ptr(),
            grad.data_ptr(), None, 0, None]
    for i in (5, 6, 7):  # target, loss, grad NULL
        bad = list(args)
        bad[i] = None
        assert lib.gcdf_train_mse(*bad) == EINVAL
    for b in (0, 101):  # batch outside [1, max_batch]
        bad = list(args)
        bad[4] = b
        assert lib.gcdf_train_mse(*bad) == EINVAL
    assert lib.gcdf_train_mse(*args) == 0
    with pytest.raises(ValueError):
        trainer.mse(params, kt, pt, yt[:50].contiguous())
    trainer.close()


def test_fused_mse_autograd_and_determinism(tr_mod):
    w = wl.weights(256, seed=42, bf16_hidden=False)
    k, p, y = batch(2048 + 37, 17)
    trainer, params, kt, pt, loss, d, g = fused_grads(tr_mod, "bf16", w, k, p, y)
    yt = torch.from_numpy(y).cuda()
    _, g2 = trainer.mse(params, kt, pt, yt)
    assert np.array_equal(g, g2.cpu().numpy())  # deterministic
    pr = params.clone().requires_grad_(True)
    lt = tr_mod.gcdf_mse(pr, kt, pt, yt, trainer)
    assert lt.dim() == 0 and float(lt.item()) == loss
    (3.0 * lt).backward()  # the upstream gradient scales the fused one
    assert torch.equal(pr.grad, 3.0 * torch.from_numpy(g).cuda())
    with pytest.raises(ValueError):
        tr_mod.gcdf_mse(pr, kt, pt, yt[:-1].contiguous(), trainer)


def test_gradient_matches_finite_differences_multi_chunk(tr_mod):
    """Central differences of the GPU's own FP32 MSE loss at the multi-chunk batch."""
    w = wl.weights(256, seed=39, bf16_hidden=False)
    k, p, y = batch(MULTI_B, 14)
    trainer, params, kt, pt, d, g = gpu_grads(tr_mod, "fp32", w, k, p, y)
    yt = torch.from_numpy(y).cuda()

    def loss(pv):
        dd = trainer.forward(pv, kt, pt).double()
        return float(((dd - yt.double()) ** 2).mean())

    # the largest components of every parameter array, so each reduction path is hit
    picks, off = [], 0
    for a in w.flat_params():
        seg = np.abs(g[off:off + a.size])
        picks += [off + int(i) for i in np.argsort(-seg)[:2]]
        off += a.size
    h = 1e-3
    for i in picks:
        pp, pm = params.clone(), params.clone()
        pp[i] += h
        pm[i] -= h
        fd = (loss(pp) - loss(pm)) / (2 * h)
        assert abs(fd - g[i]) <= 2e-3 * abs(g[i]) + 1e-5, (i, fd, g[i])


def test_backward_is_deterministic(tr_mod):
    w = wl.weights(256, seed=32, bf16_hidden=False)
    k, p, y = batch(2048 + 37, 4)
    trainer, params, kt, pt, d, g1 = gpu_grads(tr_mod, "bf16", w, k, p, y)
    gd = (2.0 * (torch.from_numpy(d).cuda() - torch.from_numpy(y).cuda()) / len(k)).contiguous()
    g2 = trainer.backward(params, kt, pt, gd).cpu().numpy()
    assert np.array_equal(g1, g2)


def test_gradient_matches_finite_differences_of_gpu_loss(tr_mod):
    w = wl.weights(256, seed=33, bf16_hidden=False)
    k, p, y = batch(512, 5)
    trainer, params, kt, pt, d, g = gpu_grads(tr_mod, "fp32", w, k, p, y)
    yt = torch.from_numpy(y).cuda()

    def loss(pv):
        dd = trainer.forward(pv, kt, pt).double()
        return float(((dd - yt.double()) ** 2).mean())

    idx = np.argsort(-np.abs(g))[:12]  # the largest components: well above FP32 noise
    h = 1e-3
    for i in idx:
        pp, pm = params.clone(), params.clone()
        pp[i] += h
        pm[i] -= h
        fd = (loss(pp) - loss(pm)) / (2 * h)
        assert abs(fd - g[i]) <= 2e-3 * abs(g[i]) + 1e-5, (i, fd, g[i])


def test_autograd_function_and_adam_reduce_the_loss(tr_mod):
    teacher = wl.weights(256, seed=34, bf16_hidden=False)
    student = wl.weights(256, seed=35, bf16_hidden=False)
    B = 4096
    k, p, noise = wl.training_batch(B, 6)
    trainer = tr_mod.Trainer(256, "bf16", max_batch=B)
    kt, pt = torch.from_numpy(k).cuda(), torch.from_numpy(p).cuda()
    with torch.no_grad():
        y = trainer.forward(tr_mod.flat_params(teacher), kt, pt) + torch.from_numpy(noise).cuda()
    params = tr_mod.flat_params(student).requires_grad_(True)
    # autograd gradient == direct backward
    d = tr_mod.gcdf_net(params, kt, pt, trainer)
    loss = ((d - y) ** 2).mean()
    loss.backward()
    gd = (2.0 * (d.detach() - y) / B).contiguous()
    direct = trainer.backward(params.detach(), kt, pt, gd)
    assert torch.equal(params.grad, direct)
    opt = tr_mod.adam(params, lr=5e-3)
    losses = [tr_mod.mse_step(params, opt, trainer, kt, pt, y).item() for _ in range(30)]
    print("loss %.4f -> %.4f" % (losses[0], losses[-1]), flush=True)
    assert losses[-1] < 0.5 * losses[0]


def test_native_adam_matches_torch_adam(tr_mod):
    """gcdf_adam_step against torch.optim.Adam (CPU, float64) over 25 steps."""
    rng = np.random.default_rng(11)
    n = 100_003
    p0 = rng.normal(size=n).astype(np.float32)
    grads = [rng.normal(scale=10.0 ** rng.uniform(-4, 1), size=n).astype(np.float32) for _ in range(25)]
    p = torch.from_numpy(p0.copy()).cuda().requires_grad_(True)
    opt = tr_mod.Adam(p, lr=5e-3, betas=(0.9, 0.999), eps=1e-8)
    ref = torch.from_numpy(p0.astype(np.float64)).requires_grad_(True)
    ropt = torch.optim.Adam([ref], lr=5e-3, betas=(0.9, 0.999), eps=1e-8, foreach=False)
    for g in grads:
        p.grad = torch.from_numpy(g).cuda()
        opt.step()
        ref.grad = torch.from_numpy(g.astype(np.float64))
        ropt.step()
    got = p.detach().cpu().numpy().astype(np.float64)
    want = ref.detach().numpy()
    # each step moves a parameter by at most ~lr; FP32 rounding of the update
    assert np.abs(got - want).max() <= 1e-5
    assert np.abs(got - p0).max() > 1e-2  # it did move


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_adam_step_with_trainer_packs_what_a_fresh_packing_gives(tr_mod, precision):
    """gcdf_train_adam_step: the parameters and moments bitwise equal to
    gcdf_adam_step's, and the loss and gradient of the next call, which reuses the
    packing it wrote, bitwise equal to a fresh trainer's (which packs the updated
    parameters itself); then three mse_step steps with and without the trainer in the
    optimiser give the same parameters."""
    w = wl.weights(256, seed=45, bf16_hidden=False)
    k, p, y = batch(1000, 20)
    kt, pt, yt = torch.from_numpy(k).cuda(), torch.from_numpy(p).cuda(), torch.from_numpy(y).cuda()
    trainer = tr_mod.Trainer(256, precision, max_batch=1000)
    a = tr_mod.flat_params(w)
    b = a.clone()
    _, g = trainer.mse(a, kt, pt, yt)
    g = g.clone()
    oa = tr_mod.Adam(a, lr=5e-3, trainer=trainer)
    ob = tr_mod.Adam(b, lr=5e-3)
    a.grad, b.grad = g, g.clone()
    oa.step()
    ob.step()
    assert torch.equal(a, b) and torch.equal(oa.m, ob.m) and torch.equal(oa.v, ob.v)
    assert trainer.packed_is_current(a)
    l1, g1 = trainer.mse(a, kt, pt, yt, reuse_packed=True)
    fresh = tr_mod.Trainer(256, precision, max_batch=1000)
    l2, g2 = fresh.mse(b, kt, pt, yt)
    assert torch.equal(l1, l2) and torch.equal(g1, g2)
    # whole steps through the autograd function
    pa = tr_mod.flat_params(w).requires_grad_(True)
    pb = tr_mod.flat_params(w).requires_grad_(True)
    sa, sb = tr_mod.adam(pa, trainer=trainer), tr_mod.adam(pb)
    for _ in range(3):
        tr_mod.mse_step(pa, sa, trainer, kt, pt, yt)
        tr_mod.mse_step(pb, sb, fresh, kt, pt, yt)
    assert torch.equal(pa, pb)
    trainer.close()
    fresh.close()


def test_packed_weights_reused_only_when_unchanged(tr_mod):
    """The autograd backward reuses the forward's packed weights; a direct backward
    with other parameters in between forces a repack (same gradients as a fresh
    trainer either way)."""
    w1 = wl.weights(256, seed=36, bf16_hidden=False)
    w2 = wl.weights(256, seed=37, bf16_hidden=False)
    k, p, y = batch(1000, 12)
    kt, pt, yt = torch.from_numpy(k).cuda(), torch.from_numpy(p).cuda(), torch.from_numpy(y).cuda()
    trainer = tr_mod.Trainer(256, "fp32", max_batch=1000)
    a = tr_mod.flat_params(w1).requires_grad_(True)
    b = tr_mod.flat_params(w2)
    d = tr_mod.gcdf_net(a, kt, pt, trainer)
    gd = (2.0 * (d.detach() - yt) / 1000).contiguous()
    trainer.backward(b, kt, pt, gd)  # packs b
    loss = ((d - yt) ** 2).mean()
    loss.backward()  # must repack a
    fresh = tr_mod.Trainer(256, "fp32", max_batch=1000)
    want = fresh.backward(a.detach(), kt, pt, gd)
    assert torch.equal(a.grad, want)
