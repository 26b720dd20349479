"""Pins of the oracle's sphere-obstacle variant (CPU only).

The primitive-aware extension (Sec. VII) feeds the network (q, p, r) for a
sphere of centre p and radius r; the network input is [p', r, a], 10 wide.
Each test fails on a plausible mistake in that variant:
  * the 10-wide forward / input gradient   -> torch autograd and jacrev;
  * the input order [p', r, a]              -> a radius column of zeros must
    reduce exactly to the pinned 9-input network with that column removed;
  * the radius passing through the base-frame motion -> invariance under a
    common rigid motion of base and sphere centres, radius unchanged;
  * the chain rule with spheres             -> central differences in every
    configuration coordinate, and in the radius against the network's own
    input gradient at [p', r, a];
  * sphere partitions                       -> the float64 geometric test
    away from the boundary.
"""
import math

import numpy as np
import pytest
import torch

from paper_2601_18548_amd import workloads as wl


def _torch_net(w: wl.Weights):
    mats = [torch.tensor(m, dtype=torch.float64) for m in w.mats]
    bias = [torch.tensor(b, dtype=torch.float64) for b in w.biases]

    def f(v):
        h = v
        for l in range(w.depth):
            h = torch.nn.functional.silu(torch.nn.functional.linear(h, mats[l], bias[l]))
        return torch.nn.functional.linear(h, mats[w.depth], bias[w.depth])[..., 0]

    return f


def _spheres(n, seed):
    r = np.random.default_rng(seed)
    c = r.uniform([-3, -3, 0], [3, 3, 1.5], (n, 3))
    return np.concatenate([c, r.uniform(0.05, 0.3, (n, 1))], 1)


def _knots(n, seed):
    r = np.random.default_rng(seed)
    return np.concatenate([r.uniform(-2, 2, (n, 2)), r.uniform(-math.pi, math.pi, (n, 7))], 1)


def test_sphere_network_matches_torch(oracle_mod):
    w = wl.weights(24, seed=31, in_dim=10)
    blob = w.to_blob()
    assert oracle_mod.in_dim(blob) == 10 and w.mats[0].shape == (24, 10)
    r = np.random.default_rng(4)
    v = np.concatenate([r.uniform(-3, 3, (48, 3)), r.uniform(0.05, 0.3, (48, 1)),
                        r.uniform(-math.pi, math.pi, (48, 6))], 1)
    d, e = oracle_mod.mlp(blob, v)
    f = _torch_net(w)
    vt = torch.tensor(v, dtype=torch.float64, requires_grad=True)
    dt = f(vt)
    (et,) = torch.autograd.grad(dt.sum(), vt)
    np.testing.assert_allclose(d, dt.detach().numpy(), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(e, et.numpy(), rtol=1e-11, atol=1e-13)
    jr = torch.func.vmap(torch.func.jacrev(f))(torch.tensor(v, dtype=torch.float64))
    np.testing.assert_allclose(e, jr.numpy(), rtol=1e-11, atol=1e-13)


def test_zero_radius_column_reduces_to_point_network(oracle_mod):
    """With W1[:, 3] = 0 the sphere network ignores r and must equal the point
    network whose W1 is the same matrix without that column, at the centres."""
    w10 = wl.weights(32, seed=12, in_dim=10)
    w10.mats[0][:, 3] = 0.0
    w9 = wl.Weights(w10.width, w10.depth, [np.delete(w10.mats[0], 3, axis=1)] + w10.mats[1:],
                    list(w10.biases), 9)
    k = wl.knots(5, 3)
    s = wl.spheres(13, 4)
    d10, J10 = oracle_mod.eval_grad(w10.to_blob(), k, s)
    d9, J9 = oracle_mod.eval_grad(w9.to_blob(), k, s[:, :3])
    assert np.array_equal(d10, d9) and np.array_equal(J10, J9)
    # and a non-zero radius column does change the result
    w10b = wl.weights(32, seed=12, in_dim=10)
    d10b, _ = oracle_mod.eval_grad(w10b.to_blob(), k, s, with_grad=False)
    assert np.max(np.abs(d10b - d9)) > 1e-3


def test_sphere_configuration_gradient_matches_central_differences(oracle_mod):
    blob = wl.weights(32, seed=13, in_dim=10).to_blob()
    k = _knots(4, 5)
    s = _spheres(6, 6)
    _, J = oracle_mod.eval_grad(blob, k, s)
    for i in range(len(k)):
        for c in range(9):
            h = 1e-6 * max(1.0, abs(k[i, c]))
            kp, km = k[i:i + 1].copy(), k[i:i + 1].copy()
            kp[0, c] += h
            km[0, c] -= h
            dp, _ = oracle_mod.eval_grad(blob, kp, s, with_grad=False)
            dm, _ = oracle_mod.eval_grad(blob, km, s, with_grad=False)
            np.testing.assert_allclose(J[i, :, c], (dp[0] - dm[0]) / (2 * h), rtol=1e-6, atol=1e-8)


def test_radius_enters_as_the_fourth_network_input(oracle_mod):
    """d/dr by central differences through the all-pairs entry equals the
    network's input gradient component 3 at [p', r, a] (p' from the pinned
    transform)."""
    blob = wl.weights(32, seed=14, in_dim=10).to_blob()
    k = _knots(3, 7)
    s = _spheres(5, 8)
    kk = np.repeat(k, len(s), axis=0)
    ss = np.tile(s, (len(k), 1))
    pp = oracle_mod.transform(kk, ss[:, :3])
    v = np.concatenate([pp, ss[:, 3:4], kk[:, 3:]], 1)
    d_v, e = oracle_mod.mlp(blob, v)
    d, _ = oracle_mod.eval_grad(blob, k, s, with_grad=False)
    np.testing.assert_allclose(d.reshape(-1), d_v, rtol=1e-14, atol=1e-14)
    h = 1e-6
    sp, sm = s.copy(), s.copy()
    sp[:, 3] += h
    sm[:, 3] -= h
    fd = (oracle_mod.eval_grad(blob, k, sp, False)[0] - oracle_mod.eval_grad(blob, k, sm, False)[0]) / (2 * h)
    np.testing.assert_allclose(fd.reshape(-1), e[:, 3], rtol=1e-6, atol=1e-8)


@pytest.mark.parametrize("phi,dx,dy", [(0.7, 0.3, -1.1), (-2.5, -0.8, 0.4)])
def test_sphere_invariance_to_common_rigid_motion(oracle_mod, phi, dx, dy):
    blob = wl.weights(32, seed=15, in_dim=10).to_blob()
    k = _knots(4, 9)
    s = _spheres(9, 10)
    d, J = oracle_mod.eval_grad(blob, k, s)
    c, sn = math.cos(phi), math.sin(phi)
    k2 = k.copy()
    k2[:, 0] = c * k[:, 0] - sn * k[:, 1] + dx
    k2[:, 1] = sn * k[:, 0] + c * k[:, 1] + dy
    k2[:, 2] = k[:, 2] + phi
    s2 = s.copy()  # the radius column is left alone
    s2[:, 0] = c * s[:, 0] - sn * s[:, 1] + dx
    s2[:, 1] = sn * s[:, 0] + c * s[:, 1] + dy
    d2, J2 = oracle_mod.eval_grad(blob, k2, s2)
    np.testing.assert_allclose(d2, d, rtol=0, atol=1e-12)
    np.testing.assert_allclose(J2[..., 2:], J[..., 2:], rtol=0, atol=1e-11)
    np.testing.assert_allclose(J2[..., 0], c * J[..., 0] - sn * J[..., 1], atol=1e-11)
    np.testing.assert_allclose(J2[..., 1], sn * J[..., 0] + c * J[..., 1], atol=1e-11)


def test_sphere_pairs_entry_agrees_with_all_pairs(oracle_mod):
    blob = wl.weights(16, seed=16, in_dim=10).to_blob()
    k = wl.knots(4, 11)
    s = wl.spheres(7, 12)
    d, J = oracle_mod.eval_grad(blob, k, s)
    ki = np.array([0, 3, 2, 1, 3])
    pi = np.array([6, 0, 4, 2, 2])
    dp, Jp = oracle_mod.eval_pairs(blob, k, s, ki, pi)
    assert np.array_equal(dp, d[ki, pi]) and np.array_equal(Jp, J[ki, pi])


def test_sphere_blob_checks(oracle_mod):
    w = wl.weights(8, seed=17, in_dim=10)
    blob = w.to_blob()
    w2 = wl.Weights.from_blob(blob)
    assert w2.in_dim == 10
    for a, b in zip(w.flat_params(), w2.flat_params()):
        assert np.array_equal(a, b)
    bad = bytearray(blob)
    bad[8:12] = (11).to_bytes(4, "little")
    with pytest.raises(ValueError):
        oracle_mod.in_dim(bytes(bad))
    with pytest.raises(ValueError):  # the obstacle width follows the blob
        oracle_mod.eval_grad(blob, wl.knots(2, 1), wl.points_uniform(3, 2))
    with pytest.raises(ValueError):  # training losses are for point networks
        oracle_mod.mse_grad(blob, np.zeros((1, 9)), np.zeros((1, 3)), np.zeros(1))


def test_sphere_partition_is_the_geometric_range_test():
    from oracle import constraints as oc

    ref = wl.trajectory(12, 21)[:, :2]
    s = wl.spheres(3000, 22)
    R = 0.9
    off, idx = oc.partition(ref, s, R)
    dist = np.hypot(s[None, :, 0].astype(np.float64) - ref[:, None, 0], s[None, :, 1].astype(np.float64) - ref[:, None, 1])
    reach = np.broadcast_to(R + s[None, :, 3].astype(np.float64), dist.shape)
    clear = np.abs(dist - reach) > 1e-4
    for i in range(len(ref)):
        got = np.zeros(len(s), bool)
        got[idx[off[i]:off[i + 1]]] = True
        assert np.array_equal(got[clear[i]], (dist[i] <= reach[i])[clear[i]])
        assert np.all(np.diff(idx[off[i]:off[i + 1]]) > 0)
    # zero radii reduce to the point partition of the centres
    s0 = s.copy()
    s0[:, 3] = 0.0
    o0, i0 = oc.partition(ref, s0, R)
    o3, i3 = oc.partition(ref, s[:, :3], R)
    assert np.array_equal(o0, o3) and np.array_equal(i0, i3)
