"""Pins of the oracle's Table I training loss and its weight gradient.

* torch float64 autograd with a double backward: the configuration gradient
  J = dF/dq is taken by torch through the base-frame transform and the network
  (create_graph=True), the four loss terms are formed from it and the total is
  differentiated again with respect to the weights -- an independent route to
  both the loss values and the gradient;
* central finite differences of the oracle's total loss on sampled weights;
* closed forms: L_grad = 0 when J* is a positive multiple of J and 4 when it is
  a negative one; L_tension = mean |J|^2; the eikonal term of a target whose
  weighted norm is known.
"""
import numpy as np
import pytest

from paper_2601_18548_amd import workloads as wl

torch = pytest.importorskip("torch")

M_DIAG = np.array([4.0, 4.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0])


def _net_torch(w):
    return [torch.tensor(a.astype(np.float64), requires_grad=True) for a in w.flat_params()]


def _forward_torch(params, q, p):
    """F(q, p) for a batch, float64, with torch ops only."""
    c, s = torch.cos(q[:, 2]), torch.sin(q[:, 2])
    ux, uy = p[:, 0] - q[:, 0], p[:, 1] - q[:, 1]
    v = torch.stack([c * ux + s * uy, -s * ux + c * uy, p[:, 2]], dim=1)
    h = torch.cat([v, q[:, 3:]], dim=1)
    n = (len(params) - 2) // 2
    for l in range(n):
        h = torch.nn.functional.silu(h @ params[2 * l].T + params[2 * l + 1])
    return (h @ params[-2].T).squeeze(1) + params[-1]


def _samples(n, seed):
    k = wl.knots(n, seed).astype(np.float64)
    p = wl.points_uniform(n, seed + 1).astype(np.float64)
    return k, p


def _targets(seed, n):
    r = np.random.default_rng(seed)
    return r.normal(size=n), r.normal(size=(n, 9))


def test_loss_and_gradient_match_torch_double_backward(oracle_mod):
    w = wl.weights(48, seed=71, bf16_hidden=False)
    n = 24
    k, p = _samples(n, 3)
    fs, Js = _targets(5, n)
    lam = np.array([5.0, 0.1, 0.01, 0.01])
    total, losses, grads = oracle_mod.table1_grad(w.to_blob(), k, p, fs, Js, M_DIAG, lam)

    params = _net_torch(w)
    q = torch.tensor(k, requires_grad=True)
    pt = torch.tensor(p)
    f = _forward_torch(params, q, pt)
    (J,) = torch.autograd.grad(f.sum(), q, create_graph=True)
    Jt = torch.tensor(Js)
    cos = (J * Jt).sum(1) / (J.norm(dim=1) * Jt.norm(dim=1))
    nm = torch.sqrt((J * J / torch.tensor(M_DIAG)).sum(1))
    L = torch.stack([((f - torch.tensor(fs)) ** 2).mean(), ((1 - cos) ** 2).mean(), ((nm - 1) ** 2).mean(),
                     (J * J).sum(1).mean()])
    tot = (torch.tensor(lam) * L).sum()
    tot.backward()
    np.testing.assert_allclose(losses, L.detach().numpy(), rtol=1e-11)
    assert total == pytest.approx(float(tot.detach()), rel=1e-11)
    for a, b in zip(grads, params):
        ref = b.grad.numpy()
        assert np.abs(a - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max())


def test_gradient_matches_finite_differences(oracle_mod):
    w = wl.weights(32, seed=72, bf16_hidden=False)
    n = 12
    k, p = _samples(n, 6)
    fs, Js = _targets(7, n)
    blob = bytearray(w.to_blob())
    _, _, grads = oracle_mod.table1_grad(bytes(blob), k, p, fs, Js, M_DIAG)
    flat = np.frombuffer(bytes(blob), dtype=np.float32, offset=32).copy()
    gflat = np.concatenate([g.ravel() for g in grads])
    rng = np.random.default_rng(8)
    idx = np.concatenate([rng.choice(len(flat), 40, replace=False), [len(flat) - 1]])  # includes b_out
    for i in idx:
        vals = []
        for sgn in (+1, -1):
            f2 = flat.copy()
            f2[i] = np.float32(flat[i] + sgn * np.float32(2.0 ** -10))
            b2 = bytes(blob[:32]) + f2.tobytes()
            vals.append((oracle_mod.table1_grad(b2, k, p, fs, Js, M_DIAG)[0], float(f2[i])))
        fd = (vals[0][0] - vals[1][0]) / (vals[0][1] - vals[1][1])
        assert abs(fd - gflat[i]) <= 1e-5 * max(1.0, abs(gflat[i])) + 1e-7, (i, fd, gflat[i])


def test_closed_form_loss_values(oracle_mod):
    w = wl.weights(32, seed=73, bf16_hidden=False)
    n = 10
    k, p = _samples(n, 9)
    d, J = oracle_mod.eval_grad(w.to_blob(), k, p)
    f = d[np.arange(n), np.arange(n)]
    Jd = J[np.arange(n), np.arange(n)]
    scale = np.random.default_rng(10).uniform(0.5, 3.0, size=(n, 1))
    _, L, _ = oracle_mod.table1_grad(w.to_blob(), k, p, f, scale * Jd, M_DIAG)
    assert L[0] == pytest.approx(0.0, abs=1e-24)              # exact value targets
    assert L[1] == pytest.approx(0.0, abs=1e-24)              # same direction
    assert L[3] == pytest.approx(np.mean(np.sum(Jd * Jd, 1)), rel=1e-12)
    nm = np.sqrt(np.sum(Jd * Jd / M_DIAG, 1))
    assert L[2] == pytest.approx(np.mean((nm - 1) ** 2), rel=1e-12)
    _, L2, _ = oracle_mod.table1_grad(w.to_blob(), k, p, f + 0.5, -Jd, M_DIAG)
    assert L2[0] == pytest.approx(0.25, rel=1e-12)
    assert L2[1] == pytest.approx(4.0, rel=1e-12)              # opposite direction
