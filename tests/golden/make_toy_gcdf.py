"""Writes toy_gcdf_512.txt: training pairs for the planar toy robot of oracle/toy.py.

Uses only the oracle.  Each row is one (knot, point) pair of the 9-wide
configuration (x, y, yaw, a1, a2, a3..a6 = 0) and a point on the floor plane
(p_z = 0): the toy GCDF value B (Definition 1, M = identity) and its configuration
gradient (the toy's base-frame gradient through the oracle's transform and chain
rule, the arm columns a3..a6 zero).  Pairs are kept only where the minimiser has
the point strictly outside the robot (signed distance > 0.05 m) and the best arm
candidate is unique (relative gap > 1e-3), so B is differentiable there and its
gradient has unit norm (Theorem 1).  Run: python tests/golden/make_toy_gcdf.py
"""
import math
import os
import sys
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
import oracle  # noqa: E402
from oracle import toy  # noqa: E402

N = 512
SEED = 2601


def candidate(i):
    r = np.random.default_rng([SEED, i])
    x, y = r.uniform(-1.0, 1.0, 2)
    yaw, a1, a2 = r.uniform(-math.pi, math.pi, 3)
    rad, ang = 1.6 * math.sqrt(r.uniform(0.0, 1.0)), r.uniform(-math.pi, math.pi)
    pb = np.array([rad * math.cos(ang), rad * math.sin(ang)])  # base-frame point
    res = toy.gcdf_base(pb, (a1, a2), w_t=1.0, tol=1e-9)
    if not (res["sdf"] > 0.05 and res["value"] > 0.05 and res["gap"] > 1e-3):
        return None
    c, s = math.cos(yaw), math.sin(yaw)
    px, py = x + c * pb[0] - s * pb[1], y + s * pb[0] + c * pb[1]
    return [x, y, yaw, a1, a2, px, py, res["value"], *res["e"]]


def main():
    rows = []
    with Pool(8) as pool:
        start = 0
        while len(rows) < N:
            got = pool.map(candidate, range(start, start + 256))
            rows += [g for g in got if g is not None]
            start += 256
    rows = np.array(rows[:N], dtype=np.float64)
    knots = np.zeros((N, 9))
    knots[:, :5] = rows[:, :5]
    points = np.zeros((N, 3))
    points[:, :2] = rows[:, 5:7]
    e = np.zeros((N, 9))  # network-input gradient [p'x, p'y, p'z, a1..a6]
    e[:, 0], e[:, 1], e[:, 3], e[:, 4] = rows[:, 8], rows[:, 9], rows[:, 10], rows[:, 11]
    J = oracle.chain(knots, points, e)
    out = np.concatenate([rows[:, :8], J[:, :5]], axis=1)
    hdr = ("planar toy GCDF training pairs (oracle/toy.py, M = identity), written by make_toy_gcdf.py\n"
           "columns: x y yaw a1 a2 px py  B  dB/dx dB/dy dB/dyaw dB/da1 dB/da2  (a3..a6 = 0, pz = 0)")
    np.savetxt(os.path.join(HERE, "toy_gcdf_512.txt"), out, fmt="%.10g", header=hdr)


if __name__ == "__main__":
    main()
