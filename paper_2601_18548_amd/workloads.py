"""Seeded synthetic inputs for the batched neural GCDF query.

This module only draws inputs: knot configurations, obstacle point clouds,
network weights (and the weight-blob byte format), serving traces and training
batches.  It holds none of the query's arithmetic (no transform, no network,
no derivative), so both the FP64 oracle and the HIP path can consume what it
produces without sharing computation.

Configuration layout of a knot (Sec. IV-A, state definition): the planar base
translation (x, y), the base yaw (first rotational coordinate), then the six
arm joints -> ``float32[K][9]`` in the order (x, y, yaw, a1..a6).

Obstacle points are stored as ``float32[Np][3]`` world coordinates, the "one
array of all obstacle coordinates" of the partition data structure (Sec. IV-A).
For the primitive-aware network (sphere obstacles with radius r, the (q, p, r)
input of the closing discussion, Sec. VII) obstacles are ``float32[Np][4]`` =
(x, y, z, r) and the network has 10 inputs [p', r, a].

All generators use numpy's PCG64 with an explicit seed.
"""
from __future__ import annotations

import math
import struct
from dataclasses import dataclass

import numpy as np

IN_DIM = 9          # point obstacles: network input [p', a]
IN_DIM_SPHERE = 10  # sphere obstacles: network input [p', r, a]
BLOB_MAGIC = b"GCDF"
BLOB_VERSION = 1
BLOB_HEADER_BYTES = 32  # magic, version, in_dim, width, depth, 3 reserved u32

# Workspace box for obstacle points, metres: [-3,3] x [-3,3] x [0,1.5].
BOX_LO = np.array([-3.0, -3.0, 0.0])
BOX_HI = np.array([3.0, 3.0, 1.5])


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


# ----------------------------------------------------------------------------
# knots and points
# ----------------------------------------------------------------------------
def knots(K: int, seed: int) -> np.ndarray:
    """K knot configurations: x,y ~ U[-2,2] m, yaw ~ U[-pi,pi], arm ~ U[-pi,pi]^6."""
    r = _rng(seed)
    xy = r.uniform(-2.0, 2.0, size=(K, 2))
    yaw = r.uniform(-math.pi, math.pi, size=(K, 1))
    arm = r.uniform(-math.pi, math.pi, size=(K, 6))
    return np.ascontiguousarray(np.concatenate([xy, yaw, arm], axis=1), dtype=np.float32)


def trajectory(N: int, seed: int) -> np.ndarray:
    """N knots along one planar base path across the workspace box: the base
    moves from x = -2.5 to 2.5 with a sinusoidal y offset, yaw along the path
    tangent, arm joints a smooth random walk.  ``float32[N][9]``; consecutive
    knots are close, so their obstacle partitions overlap."""
    r = _rng(seed)
    s = np.linspace(0.0, 1.0, N)
    amp, phase = r.uniform(0.5, 1.5), r.uniform(-math.pi, math.pi)
    x = -2.5 + 5.0 * s
    y = amp * np.sin(2 * math.pi * s + phase)
    dy = amp * 2 * math.pi * np.cos(2 * math.pi * s + phase) / 5.0
    yaw = np.arctan2(dy, np.ones_like(dy))
    arm = np.cumsum(r.normal(0.0, 0.1, size=(N, 6)), axis=0) + r.uniform(-1.0, 1.0, size=6)
    return np.concatenate([x[:, None], y[:, None], yaw[:, None], arm], axis=1).astype(np.float32)


def points_uniform(Np: int, seed: int) -> np.ndarray:
    """Np points uniform in the workspace box."""
    r = _rng(seed)
    return np.ascontiguousarray(r.uniform(BOX_LO, BOX_HI, size=(Np, 3)), dtype=np.float32)


def points_patches(Np: int, seed: int, n_patches: int = 6, frac: float = 0.7,
                   sigma: float = 0.005) -> np.ndarray:
    """Point cloud with 70% of the points on axis-aligned planar patches.

    Each patch: a normal axis drawn uniformly from {x, y, z}, a centre uniform
    in the box, in-plane side lengths U[0.2, 1.0] m clipped to the box, points
    uniform on that rectangle plus isotropic Gaussian noise (sigma = 5 mm).
    round(frac*Np) patch points are split evenly over the patches (remainder
    to the first ones); the rest are uniform in the box.  The result is
    shuffled with the same generator.
    """
    r = _rng(seed)
    n_on = int(round(frac * Np))
    per = [n_on // n_patches + (1 if i < n_on % n_patches else 0) for i in range(n_patches)]
    chunks = []
    for i in range(n_patches):
        axis = int(r.integers(0, 3))
        centre = r.uniform(BOX_LO, BOX_HI)
        side = r.uniform(0.2, 1.0, size=2)
        lo = centre.copy()
        hi = centre.copy()
        in_plane = [a for a in range(3) if a != axis]
        for s, a in zip(side, in_plane):
            lo[a] = max(BOX_LO[a], centre[a] - 0.5 * s)
            hi[a] = min(BOX_HI[a], centre[a] + 0.5 * s)
        pts = r.uniform(lo, hi, size=(per[i], 3))
        pts[:, axis] = centre[axis]
        pts += r.normal(0.0, sigma, size=pts.shape)
        chunks.append(pts)
    chunks.append(r.uniform(BOX_LO, BOX_HI, size=(Np - n_on, 3)))
    allp = np.concatenate(chunks, axis=0)
    allp = allp[r.permutation(Np)]
    return np.ascontiguousarray(allp, dtype=np.float32)


# ----------------------------------------------------------------------------
# weights
# ----------------------------------------------------------------------------
def round_to_bf16_grid(a: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 value (ties to even), kept as float32."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).reshape(a.shape)


@dataclass
class Weights:
    """Distance-MLP parameters, float32, out x in row-major (Sec. III-C network)."""
    width: int
    depth: int
    mats: list  # [W1 (W x in_dim), W2..W_depth (W x W), w_out (1 x W)]
    biases: list  # [b1 (W), ..., b_depth (W), b_out (1)]
    in_dim: int = IN_DIM

    def to_blob(self) -> bytes:
        hdr = BLOB_MAGIC + struct.pack("<7I", BLOB_VERSION, self.in_dim, self.width, self.depth, 0, 0, 0)
        assert len(hdr) == BLOB_HEADER_BYTES
        parts = [hdr]
        for m, b in zip(self.mats, self.biases):
            parts.append(np.ascontiguousarray(m, dtype="<f4").tobytes())
            parts.append(np.ascontiguousarray(b, dtype="<f4").tobytes())
        return b"".join(parts)

    @staticmethod
    def from_blob(blob: bytes) -> "Weights":
        if blob[:4] != BLOB_MAGIC:
            raise ValueError("bad weight blob magic")
        version, in_dim, width, depth = struct.unpack("<4I", blob[4:20])
        if version != BLOB_VERSION or in_dim not in (IN_DIM, IN_DIM_SPHERE):
            raise ValueError("unsupported weight blob")
        off = BLOB_HEADER_BYTES
        mats, biases = [], []
        dims = [in_dim] + [width] * depth + [1]
        for li in range(depth + 1):
            fi, fo = dims[li], dims[li + 1]
            m = np.frombuffer(blob, dtype="<f4", count=fo * fi, offset=off).reshape(fo, fi).copy()
            off += 4 * fo * fi
            b = np.frombuffer(blob, dtype="<f4", count=fo, offset=off).copy()
            off += 4 * fo
            mats.append(m)
            biases.append(b)
        if off != len(blob):
            raise ValueError("weight blob size mismatch")
        return Weights(width, depth, mats, biases, in_dim)

    def flat_params(self) -> list:
        out = []
        for m, b in zip(self.mats, self.biases):
            out += [m, b]
        return out


def weights(width: int, seed: int, depth: int = 4, bf16_hidden: bool = True, in_dim: int = IN_DIM) -> Weights:
    """He-normal weights N(0, 2/fan_in) for every layer, biases U(+-1/sqrt(fan_in)).

    Draw order W1, b1, W2, b2, ..., w_out, b_out from one PCG64 stream.  The
    square hidden matrices W2..W_depth are rounded to the bfloat16 grid so that
    a BF16 matrix-core path multiplies by exactly the same weights.  in_dim 10
    gives the sphere-obstacle network (W1 columns p'x, p'y, p'z, r, a1..a6).
    """
    if in_dim not in (IN_DIM, IN_DIM_SPHERE):
        raise ValueError("in_dim must be 9 or 10")
    r = _rng(seed)
    dims = [in_dim] + [width] * depth + [1]
    mats, biases = [], []
    for li in range(depth + 1):
        fi, fo = dims[li], dims[li + 1]
        m = r.normal(0.0, math.sqrt(2.0 / fi), size=(fo, fi)).astype(np.float32)
        bnd = 1.0 / math.sqrt(fi)
        b = r.uniform(-bnd, bnd, size=fo).astype(np.float32)
        if bf16_hidden and 1 <= li <= depth - 1:
            m = round_to_bf16_grid(m)
        mats.append(m)
        biases.append(b)
    return Weights(width, depth, mats, biases, in_dim)


def spheres(Np: int, seed: int, r_lo: float = 0.05, r_hi: float = 0.25) -> np.ndarray:
    """Np sphere obstacles ``float32[Np][4]`` = (x, y, z, r): centres from the
    patch cloud of the same seed (points_patches), radii U[r_lo, r_hi] m from a
    second PCG64 stream (seed + 7919)."""
    c = points_patches(Np, seed)
    rad = _rng(seed + 7919).uniform(r_lo, r_hi, size=(Np, 1))
    return np.ascontiguousarray(np.concatenate([c, rad.astype(np.float32)], axis=1), dtype=np.float32)


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------
@dataclass
class QueryWorkload:
    name: str
    K: int
    Np: int
    width: int
    precision: str  # "fp32" | "bf16" | "bf16x2" | "bf16x2_f16"
    knots: np.ndarray
    points: np.ndarray
    weights: Weights


def workload(name: str, seed: int = 0) -> QueryWorkload:
    """The fixed query workloads.

    small   : 16 knots x 64 uniform points, width 256 (1,024 pairs)
    fp32    : 64 knots x 4,096 patch points, width 256, FP32 (262,144 pairs)
    bf16    : 128 knots x 16,384 patch points, width 512, BF16 matrix cores (split
              activations forward, FP16 reverse sweep) (2,097,152 pairs)
    sphere  : the bf16 shape with sphere obstacles (patch-cloud centres, radii
              U[0.05, 0.25] m) and the 10-input network [p', r, a]
    """
    if name == "small":
        return QueryWorkload(name, 16, 64, 256, "fp32", knots(16, seed + 1),
                             points_uniform(64, seed + 2), weights(256, seed + 3))
    if name == "fp32":
        return QueryWorkload(name, 64, 4096, 256, "fp32", knots(64, seed + 1),
                             points_patches(4096, seed + 2), weights(256, seed + 3))
    if name == "bf16":
        return QueryWorkload(name, 128, 16384, 512, "bf16x2_f16", knots(128, seed + 1),
                             points_patches(16384, seed + 2), weights(512, seed + 3))
    if name == "sphere":
        return QueryWorkload(name, 128, 16384, 512, "bf16x2_f16", knots(128, seed + 1),
                             spheres(16384, seed + 2), weights(512, seed + 3, in_dim=IN_DIM_SPHERE))
    raise KeyError(name)


# ----------------------------------------------------------------------------
# serving trace
# ----------------------------------------------------------------------------
@dataclass
class Request:
    arrival_s: float
    K: int
    Np: int
    seed: int


def serving_trace(n_requests: int, rate_hz: float, seed: int,
                  k_range=(16, 256), np_range=(512, 32768)) -> list:
    """Poisson arrivals (exponential gaps, mean 1/rate); K and Np uniform integers, inclusive."""
    r = _rng(seed)
    gaps = r.exponential(1.0 / rate_hz, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    Ks = r.integers(k_range[0], k_range[1] + 1, size=n_requests)
    Nps = r.integers(np_range[0], np_range[1] + 1, size=n_requests)
    return [Request(float(t[i]), int(Ks[i]), int(Nps[i]), int(seed + 1000 + i)) for i in range(n_requests)]


def request_inputs(req: Request) -> tuple:
    return knots(req.K, req.seed), points_patches(req.Np, req.seed + 7)


# ----------------------------------------------------------------------------
# training batch
# ----------------------------------------------------------------------------
def training_batch(B: int, seed: int, noise_sigma: float = 1e-3) -> tuple:
    """B (configuration, point) samples drawn as the small workload, plus target noise.

    Returns (knots[B][9], points[B][3], noise[B]); the targets are a teacher
    network's distances plus ``noise`` (standard deviation ``noise_sigma``).
    """
    r = _rng(seed)
    k = knots(B, int(r.integers(0, 2**31)))
    p = points_uniform(B, int(r.integers(0, 2**31)))
    noise = r.normal(0.0, noise_sigma, size=B).astype(np.float32)
    return k, p, noise
