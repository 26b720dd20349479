"""GCDF structure (Theorem 1) on a brute-force planar robot, through the
oracle's own base-frame transform and chain rule (CPU only).

For pairs strictly outside the robot with a unique minimiser:
  * weighted eikonal: |J|_{M^-1} = 1 with M = diag(w_t, w_t, 1, 1, 1);
  * single-step projection: q - f M^-1 J lands on the zero set;
  * the toy's minimiser gradient equals central differences of its value;
  * value and gradient are invariant to a common rigid motion of base and point.
Pairs whose minimiser is ambiguous (near-equal candidates) or which sit too
close to the zero set are skipped, as the gradient is not unique there.
"""
import math

import numpy as np
import pytest

from oracle import toy

N_PAIRS = 10


def _pairs(seed, n):
    r = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        q = np.array([r.uniform(-1, 1), r.uniform(-1, 1), r.uniform(-math.pi, math.pi),
                      r.uniform(-math.pi, math.pi), r.uniform(-math.pi, math.pi)])
        p = np.array([r.uniform(-2.5, 2.5), r.uniform(-2.5, 2.5)])
        out.append((q, p))
    return out


def _knot9(q):
    return np.array([[q[0], q[1], q[2], q[3], q[4], 0, 0, 0, 0]])


def _evaluate(oracle_mod, q, p, w_t):
    k9 = _knot9(q)
    p3 = np.array([[p[0], p[1], 0.0]])
    pp = oracle_mod.transform(k9, p3)[0]
    res = toy.gcdf_base(pp[:2], q[3:5], w_t)
    e9 = np.zeros((1, 9))
    e9[0, 0], e9[0, 1], e9[0, 3], e9[0, 4] = res["e"]
    J = oracle_mod.chain(k9, p3, e9)[0]
    return res, np.array([J[0], J[1], J[2], J[3], J[4]])


def _usable(res):
    return res["value"] > 0.05 and res["gap"] > 1e-3 and res["sdf"] > 1e-4


@pytest.mark.parametrize("w_t", [1.0, 4.0])
def test_weighted_eikonal_and_single_step_projection(oracle_mod, w_t):
    minv = np.array([1 / w_t, 1 / w_t, 1.0, 1.0, 1.0])
    used = 0
    for q, p in _pairs(int(w_t * 10), 3 * N_PAIRS):
        if toy.sdf_world(p, q) <= 0.05:
            continue
        res, J = _evaluate(oracle_mod, q, p, w_t)
        if not _usable(res):
            continue
        used += 1
        f = res["value"]
        # the oracle's projection routine on the 9-coordinate layout (unused arm joints zero)
        m9 = np.r_[w_t, w_t, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0]
        qz9, eik = oracle_mod.project(_knot9(q)[0], f, np.r_[J, 0, 0, 0, 0], m9)
        assert eik == pytest.approx(1.0, abs=1e-9)  # Theorem 1 (1)
        qz = qz9[:5]  # Theorem 1 (2)
        assert np.array_equal(qz9[5:], np.zeros(4))
        assert math.sqrt(np.sum(minv * J * J)) == pytest.approx(1.0, abs=1e-9)
        assert abs(toy.sdf_world(p, qz)) < 1e-8
        # the projected arm lands exactly on the grid minimiser
        np.testing.assert_allclose(toy.wrap(qz[3:5] - np.array(res["arm"])), 0.0, atol=1e-12)
        if used >= N_PAIRS:
            break
    assert used >= 5


def test_toy_gradient_matches_central_differences():
    r = np.random.default_rng(2)
    checked = 0
    while checked < 5:
        pxy = r.uniform(-2.5, 2.5, 2)
        a = r.uniform(-math.pi, math.pi, 2)
        res = toy.gcdf_base(pxy, a, 4.0)
        if not _usable(res) or toy.sdf_base(pxy[0], pxy[1], a[0], a[1]) <= 0.05:
            continue
        h = 1e-6
        fd = []
        for i in range(4):
            x = np.concatenate([pxy, a])
            xp, xm = x.copy(), x.copy()
            xp[i] += h
            xm[i] -= h
            fd.append((toy.gcdf_value(xp[:2], xp[2:], 4.0) - toy.gcdf_value(xm[:2], xm[2:], 4.0)) / (2 * h))
        np.testing.assert_allclose(res["e"], fd, atol=1e-6)
        checked += 1


def test_toy_invariance_to_common_rigid_motion(oracle_mod):
    used = 0
    for q, p in _pairs(5, 3 * N_PAIRS):
        if toy.sdf_world(p, q) <= 0.05:
            continue
        res, J = _evaluate(oracle_mod, q, p, 1.0)
        if not _usable(res):
            continue
        phi, dx, dy = 1.1, -0.4, 0.9
        c, s = math.cos(phi), math.sin(phi)
        q2 = q.copy()
        q2[0], q2[1] = c * q[0] - s * q[1] + dx, s * q[0] + c * q[1] + dy
        q2[2] = q[2] + phi
        p2 = np.array([c * p[0] - s * p[1] + dx, s * p[0] + c * p[1] + dy])
        res2, J2 = _evaluate(oracle_mod, q2, p2, 1.0)
        assert res2["value"] == pytest.approx(res["value"], abs=1e-10)
        np.testing.assert_allclose(J2[2:], J[2:], atol=1e-8)
        np.testing.assert_allclose(J2[:2], [c * J[0] - s * J[1], s * J[0] + c * J[1]], atol=1e-8)
        used += 1
        if used >= 5:
            break
    assert used >= 3


def test_toy_sdf_closed_forms():
    # on the body disc boundary, and on the tip of a straight arm
    assert toy.sdf_base(0.25, 0.0, math.pi / 2, 0.0) == pytest.approx(0.0, abs=1e-15)
    assert toy.sdf_base(1.1 + 0.05, 0.0, 0.0, 0.0) == pytest.approx(0.0, abs=1e-15)
    assert toy.sdf_base(2.0, 0.0, 0.0, 0.0) == pytest.approx(2.0 - 1.1 - 0.05, abs=1e-15)
    # translation-only distance: with the arm pointing away, a point beyond the
    # disc along -x is reached by moving the base only, so f = sqrt(w_t) * sdf
    res = toy.gcdf_base(np.array([-1.0, 0.0]), np.array([0.0, 0.0]), 4.0)
    assert res["value"] <= 2.0 * (1.0 - 0.25) + 1e-12
