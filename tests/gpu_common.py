"""Shared helpers of the GPU parity tests: seeded inputs, oracle results
(computed only from those inputs, never from HIP outputs), packing and masks."""
from __future__ import annotations

import functools

import numpy as np

from oracle import calib, eig as oeig, gx as ogx, lagkernel, maps as omaps, nullspace, support
from oracle import pipeline as opipe
from synth import as_device_input, workloads


def packed_upper(G: np.ndarray) -> np.ndarray:
    """[N, Q, Q] -> [Q(Q+1)/2, N], entry (p, q), p <= q, row-major order."""
    Q = G.shape[1]
    iu = np.triu_indices(Q)
    return np.ascontiguousarray(G[:, iu[0], iu[1]].T)


def unpack_upper(Gp: np.ndarray, Q: int) -> np.ndarray:
    N = Gp.shape[1]
    iu = np.triu_indices(Q)
    G = np.zeros((N, Q, Q), dtype=np.complex128)
    G[:, iu[0], iu[1]] = Gp.T
    G[:, iu[1], iu[0]] = np.conj(Gp.T)
    return G


def lowres_mask(c_lr: np.ndarray, rho: np.ndarray, G: np.ndarray | None, erode: int = 1):
    """Voxels where the map is defined up to phase (Sec. II): the coil-combined
    apodized image |m| >= 1e-3 max|m| and, when G is given, a relative
    eigen-gap (lambda_2 - lambda_1)/|Lambda| >= 1e-3 is left for the caller.
    Eroded by `erode` low-res voxels."""
    from scipy.ndimage import binary_erosion
    m = np.abs(np.sum(np.conj(c_lr) * rho, axis=0))
    good = m >= 1e-3 * m.max()
    if erode:
        good = binary_erosion(good, iterations=erode)
    return good


def output_mask(lr_mask: np.ndarray, grid_out) -> np.ndarray:
    """Output voxels whose nearest low-res voxel is in lr_mask."""
    idx = []
    for n_lr, n_out in zip(lr_mask.shape, grid_out):
        x = (np.arange(n_out) - n_out // 2) / n_out
        idx.append(np.round(x * n_lr + n_lr // 2).astype(int) % n_lr)
    return lr_mask[np.ix_(*idx)]


@functools.lru_cache(maxsize=None)
def scan_inputs(name: str):
    w = workloads.ALL[name]
    sc = w.scan(keep_kspace=False)
    return w, as_device_input(sc.acs)


@functools.lru_cache(maxsize=None)
def oracle_full(name: str):
    """Oracle pipeline on the complex64 ACS (widened to complex128)."""
    w, acs = scan_inputs(name)
    return opipe.estimate(acs.astype(np.complex128), w.radius, w.grid_lr, w.grid)


@functools.lru_cache(maxsize=None)
def oracle_gram_split(name: str):
    """Oracle Gram, its complex64 rounding (the GPU nullspace input) and the
    FP64 split of that rounded matrix."""
    w, acs = scan_inputs(name)
    lam = support.kernel_support(w.D, w.radius)
    lags = support.difference_set(lam)
    gram = calib.gram_from_lags(calib.correlation_lags(acs.astype(np.complex128), lags), lam, lags)
    g32 = gram.astype(np.complex64)
    sp = nullspace.split_from_gram(g32.astype(np.complex128))
    return lam, lags, gram, g32, sp


def sampled_points(grid, count, seed):
    rng = np.random.default_rng(seed)
    N = int(np.prod(grid))
    idx = np.sort(rng.choice(N, size=min(count, N), replace=False))
    return idx, ogx.grid_points(grid)[idx]


def rel(a, b, scale):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / scale)


__all__ = ["packed_upper", "unpack_upper", "lowres_mask", "output_mask", "scan_inputs",
           "oracle_full", "oracle_gram_split", "sampled_points", "rel", "calib", "oeig", "ogx",
           "lagkernel", "omaps", "nullspace", "support"]
