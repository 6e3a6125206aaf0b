"""Seeded synthetic particle sets.

This module holds no arithmetic of the method: it only draws positions and
charges.  It is the one module that both the oracle's tests and the GPU path's
tests and benchmark use.

Workloads follow the paper's synthetic sets (Sec. 4.3 and Sec. 6): particles
uniform in the unit cube, or on the unit sphere (a two-dimensional set in
R^3), with charges uniform in [-1, 1).  Generator: numpy PCG64,
``default_rng(seed)``; positions are drawn first, then charges, from the same
stream.
"""
from __future__ import annotations

import numpy as np


def uniform_cube(n: int, seed: int):
    """n positions uniform in [0,1)^3 and charges uniform in [-1,1)."""
    rng = np.random.default_rng(seed)
    pos = rng.random((n, 3))
    q = rng.uniform(-1.0, 1.0, n)
    return pos, q


def sphere_surface(n: int, seed: int, jitter: float = 1e-3):
    """n positions uniform on the unit sphere centred at the origin with radius
    1 + jitter*U(-1,1), and charges uniform in [-1,1)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    r = 1.0 + jitter * rng.uniform(-1.0, 1.0, n)
    pos = v * r[:, None]
    q = rng.uniform(-1.0, 1.0, n)
    return pos, q


def make(kind: str, n: int, seed: int):
    if kind == "cube":
        return uniform_cube(n, seed)
    if kind == "sphere":
        return sphere_surface(n, seed)
    raise ValueError(f"unknown workload kind {kind!r}")


# The benchmark configurations: (kind, N, height, order, seed).
CONFIGS = {
    "cube20k_h4_p5": ("cube", 20_000, 4, 5, 1001),
    "cube1m_h6_p7": ("cube", 1_000_000, 6, 7, 1002),
    "sphere10m_h8_p7": ("sphere", 10_000_000, 8, 7, 1003),
    "cube30m_h9_p10": ("cube", 30_000_000, 9, 10, 1005),
    # the 30M configuration's density twin: the same 1.79 particles per
    # leaf slot (468,750 / 8^6) at order 10, small enough for the oracle
    "cube469k_h7_p10": ("cube", 468_750, 7, 10, 1005),
}

# Compressed-M2L tolerance a configuration runs at where it is not the
# library's default (10^-order): the 30M order-10 cube and its twin at the
# largest tolerance whose compressed mixed result stays within half the
# 1e-6 gate of FP64 on the twin (measured 3.5e-7 at 2e-7, 6.2e-7 at 3e-7).
SVD_TOL = {"cube30m_h9_p10": 2e-7, "cube469k_h7_p10": 2e-7}
