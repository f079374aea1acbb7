"""Quality metrics (oracle; test infrastructure).

Sec. III-E: the normalized projection residual projects the fully sampled
multichannel images onto the span of the estimated maps at every voxel and
reports ||residual||_2 / ||data||_2.  Because maps are defined only up to a
per-voxel complex scale (Sec. II), map-to-map comparisons use the
gauge-invariant distance e(x) = sqrt(max(0, 2 - 2 |c_ref(x)^H c(x)|)) between
unit vectors.
"""
from __future__ import annotations

import numpy as np


def projection_residual(coil_images: np.ndarray, maps: np.ndarray) -> float:
    """coil_images, maps: [Q, *grid]."""
    d = np.asarray(coil_images, dtype=np.complex128)
    c = np.asarray(maps, dtype=np.complex128)
    cc = np.sum(np.abs(c) ** 2, axis=0)
    proj = np.sum(np.conj(c) * d, axis=0)
    coef = np.zeros_like(proj)
    ok = cc > 0
    coef[ok] = proj[ok] / cc[ok]
    res = d - c * coef[None]
    return float(np.sqrt(np.sum(np.abs(res) ** 2) / np.sum(np.abs(d) ** 2)))


def unit(c: np.ndarray, axis: int = 0) -> np.ndarray:
    n = np.sqrt(np.sum(np.abs(c) ** 2, axis=axis, keepdims=True))
    return np.where(n > 0, c / np.where(n > 0, n, 1), 0)


def map_error(c_ref: np.ndarray, c: np.ndarray, axis: int = 0) -> np.ndarray:
    """Per-voxel gauge-invariant distance between the unit-normalised maps.

    Equal to sqrt(2 - 2 |a^H b|) for unit a, b, evaluated as the norm of the
    phase-aligned difference ||a - e^{i phi} b|| (e^{i phi} = phase of b^H a),
    which has no cancellation for nearly equal vectors."""
    a = unit(np.asarray(c_ref, dtype=np.complex128), axis)
    b = unit(np.asarray(c, dtype=np.complex128), axis)
    ip = np.sum(np.conj(b) * a, axis=axis, keepdims=True)
    mag = np.abs(ip)
    ph = np.where(mag > 0, ip / np.where(mag > 0, mag, 1), 1)
    return np.sqrt(np.sum(np.abs(a - ph * b) ** 2, axis=axis))
