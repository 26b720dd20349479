"""The toy-GCDF training fixture (tests/golden/toy_gcdf_512.txt, written by
make_toy_gcdf.py from oracle/toy.py): every stored configuration gradient has
unit norm (Theorem 1 with M = identity), every value is positive, and a few rows
recomputed from the toy and the oracle's transform agree."""
import math
import os

import numpy as np

import oracle
from oracle import toy

FIX = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "toy_gcdf_512.txt")


def test_fixture_gradients_are_unit_and_values_positive():
    a = np.loadtxt(FIX)
    assert a.shape == (512, 13)
    assert np.all(a[:, 7] > 0.05)
    assert np.abs(np.linalg.norm(a[:, 8:13], axis=1) - 1.0).max() < 1e-8


def test_fixture_rows_recompute():
    a = np.loadtxt(FIX)
    for row in a[[0, 100, 511]]:
        x, y, yaw, a1, a2, px, py = row[:7]
        knots = np.zeros((1, 9))
        knots[0, :5] = row[:5]
        pts = np.array([[px, py, 0.0]])
        pb = oracle.transform(knots, pts)[0, :2]
        res = toy.gcdf_base(pb, (a1, a2), w_t=1.0, tol=1e-9)
        assert abs(res["value"] - row[7]) < 1e-8
        e = np.zeros((1, 9))
        e[0, [0, 1, 3, 4]] = res["e"]
        J = oracle.chain(knots, pts, e)[0, :5]
        assert np.abs(J - row[8:13]).max() < 1e-6
        assert math.isfinite(res["gap"])
