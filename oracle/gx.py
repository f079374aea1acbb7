"""Per-voxel Q x Q matrices G(x) (oracle; test infrastructure).

Eq. (15): h_r(x, q) = sum_{n in Lambda} h_r[n, q] e^{+i 2 pi n.x};
Eq. (19): [H(x)]_rq = h_r(x, q);  Eq. (23): G(x) = H(x)^H H(x).
Eq. (24) expands G(x) into the double sum over (s, t) and Eq. (26) into a sum
over lags m of K_pq[m] e^{-i 2 pi m.x}.  All three forms are given here; the
tests pin them against each other.

Grid positions follow x_a = (a - floor(N/2)) / N per dimension.
"""
from __future__ import annotations

import numpy as np


def grid_points(grid) -> np.ndarray:
    """[prod(grid), D] positions of a centred grid, last dimension fastest."""
    axes = [(np.arange(n) - n // 2) / float(n) for n in grid]
    mesh = np.meshgrid(*axes, indexing="ij")
    return np.stack([m.reshape(-1) for m in mesh], axis=1)


def filters_at(h: np.ndarray, lam: np.ndarray, x: np.ndarray, Q: int) -> np.ndarray:
    """H(x) for every x: [Nx, R, Q] with H[x, r, q] = h_r(x, q) (Eq. 15)."""
    L = len(lam)
    E = np.exp(2j * np.pi * (x @ lam.T))           # [Nx, L], e^{+i2pi n.x}
    hr = np.asarray(h).reshape(Q, L, -1)            # [q, i, r]
    return np.einsum("xi,qir->xrq", E, hr)


def gx_from_filters(h, lam, x, Q) -> np.ndarray:
    """G(x) = H(x)^H H(x) (Eq. 23), [Nx, Q, Q]."""
    H = filters_at(h, lam, x, Q)
    return np.einsum("xrp,xrq->xpq", H.conj(), H)


def gx_eq24(h, lam, x, Q) -> np.ndarray:
    """G(x) by the double sum of Eq. (24), looping over (s, t)."""
    L = len(lam)
    hr = np.asarray(h).reshape(Q, L, -1)            # [q, i, r]
    out = np.zeros((len(x), Q, Q), dtype=np.complex128)
    for s in range(L):
        for t in range(L):
            coef = np.einsum("pr,qr->pq", hr[:, t, :].conj(), hr[:, s, :])
            ph = np.exp(2j * np.pi * (x @ (lam[s] - lam[t])))
            out += ph[:, None, None] * coef[None]
    return out


def gx_from_lag_kernel(K: np.ndarray, lags: np.ndarray, x: np.ndarray,
                       chunk: int = 4096) -> np.ndarray:
    """G_pq(x) = sum_m K_pq[m] e^{-i 2 pi m.x} (Eq. 26), [Nx, Q, Q]."""
    Q = K.shape[0]
    out = np.empty((len(x), Q, Q), dtype=np.complex128)
    Kf = K.reshape(Q * Q, -1)
    for a in range(0, len(x), chunk):
        E = np.exp(-2j * np.pi * (x[a:a + chunk] @ lags.T))   # [nx, L]
        out[a:a + chunk] = (E @ Kf.T).reshape(-1, Q, Q)
    return out


def espirit_operator(G: np.ndarray, bound: float) -> np.ndarray:
    """ESPIRiT's per-voxel operator B(x) = I - G(x)/|Lambda| (Eq. 20).

    Its eigenvector for the largest eigenvalue is the nullspace method's map;
    [Nx, Q, Q]."""
    G = np.asarray(G, dtype=np.complex128)
    Q = G.shape[-1]
    return np.eye(Q)[None] - G / float(bound)
