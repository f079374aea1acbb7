"""Kernel support Lambda and its difference set (oracle; test infrastructure).

Sec. IV-B: PISCO replaces the rectangular support {n : ||n||_inf <= tau} by
the ellipsoidal one {n in Z^D : ||n||_2 <= tau}.  The order of the points is
a convention of this repository: lexicographic, first coordinate slowest and
last coordinate fastest, matching [z][y][x] array storage.
"""
from __future__ import annotations

import itertools

import numpy as np


def kernel_support(D: int, radius: float, shape: str = "ellipsoid") -> np.ndarray:
    """Integer offsets n in Lambda, shape [|Lambda|, D], lexicographic order.

    shape="ellipsoid": ||n||_2 <= radius (Sec. IV-B, inclusive boundary).
    shape="rectangle": ||n||_inf <= floor(radius) (the conventional support
    the paper compares against in Sec. III-C)."""
    if D < 1:
        raise ValueError("D must be >= 1")
    r = int(np.floor(radius))
    pts = []
    for n in itertools.product(range(-r, r + 1), repeat=D):
        if shape == "rectangle" or sum(v * v for v in n) <= radius * radius:
            pts.append(n)
    return np.array(pts, dtype=np.int64).reshape(-1, D)


def difference_set(lam: np.ndarray) -> np.ndarray:
    """All distinct n_i - n_j for n_i, n_j in Lambda, lexicographic order."""
    diffs = {tuple(int(v) for v in (a - b)) for a in lam for b in lam}
    return np.array(sorted(diffs), dtype=np.int64).reshape(-1, lam.shape[1])


def index_of(rows: np.ndarray) -> dict:
    """Map from an offset tuple to its row index."""
    return {tuple(int(v) for v in r): i for i, r in enumerate(rows)}
