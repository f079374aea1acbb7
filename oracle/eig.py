"""Per-voxel smallest eigenvector of G(x) (oracle; test infrastructure).

Sec. III-D step 4: the map value c(x) is the right singular vector of H(x)
for the smallest singular value, i.e. the eigenvector of G(x) = H^H H for its
smallest eigenvalue.  Sec. IV-E replaces the per-voxel SVD by power iteration
run for all voxels at once (10 iterations in the paper's experiments).

Power iteration converges to the eigenvector of the LARGEST eigenvalue, so it
is run on the shifted matrix Gs(x) = |Lambda| I - G(x).  The shift is exact:
G(x) = Phi(x)^H conj(W) Phi(x) with W an orthogonal projector and
Phi^H Phi = |Lambda| I, so 0 <= G(x) <= |Lambda| I and the top eigenvector of
Gs is the bottom eigenvector of G.  Gs is |Lambda| B(x) of Eq. (20).

Initial vector (not stated in the paper; this repository's reading): e_q* with
q* the index of the smallest diagonal entry of G(x), lowest index on ties.
"""
from __future__ import annotations

import numpy as np


def smallest_exact(G: np.ndarray):
    """numpy eigh per voxel: (lambda_min [N], c [N, Q], lambda_2 [N])."""
    w, V = np.linalg.eigh(np.asarray(G, dtype=np.complex128))
    return w[:, 0], V[:, :, 0], w[:, 1]


def smallest_set(G: np.ndarray, M: int):
    """The M smallest eigenpairs per voxel (numpy eigh): one set of maps per
    small eigenvalue when the field of view is too small for the object
    (Sec. III-B footnote).  Returns (lambda [N, M] ascending, c [N, Q, M])."""
    w, V = np.linalg.eigh(np.asarray(G, dtype=np.complex128))
    return w[:, :M], V[:, :, :M]


def rayleigh(G: np.ndarray, c: np.ndarray):
    """Rayleigh quotient and residual of given vectors (Sec. IV-E check).

    G: [N, Q, Q] Hermitian, c: [N, Q].  Each c is normalised first; returns
    (lambda = c^H G c [N], ||G c - lambda c||_2 [N])."""
    G = np.asarray(G, dtype=np.complex128)
    c = np.asarray(c, dtype=np.complex128)
    c = c / np.linalg.norm(c, axis=1, keepdims=True)
    Gc = np.einsum("xpq,xq->xp", G, c)
    lam = np.real(np.einsum("xp,xp->x", c.conj(), Gc))
    return lam, np.linalg.norm(Gc - lam[:, None] * c, axis=1)


def initial_index(G: np.ndarray) -> np.ndarray:
    """q* = argmin_q G_qq(x) (first index on ties)."""
    return np.argmin(np.real(np.einsum("xqq->xq", G)), axis=1)


def power_iteration(G: np.ndarray, bound: float, n_iter: int = 10,
                    tol: float | None = None, max_iter: int = 100,
                    v0: np.ndarray | None = None):
    """FP64 power iteration v <- Gs v / ||Gs v|| with Gs = bound I - G.

    Fixed mode (tol None): exactly n_iter steps.  Tolerance mode: step until
    ||G c - lambda c|| <= tol * bound or max_iter steps, per voxel.
    Returns (c [N, Q] unit norm, lambda = c^H G c [N], residual [N],
    iterations [N])."""
    G = np.asarray(G, dtype=np.complex128)
    N, Q, _ = G.shape
    if v0 is None:
        v = np.zeros((N, Q), dtype=np.complex128)
        v[np.arange(N), initial_index(G)] = 1.0
    else:
        v = np.asarray(v0, dtype=np.complex128).copy()
        v /= np.linalg.norm(v, axis=1, keepdims=True)
    Gs = bound * np.eye(Q)[None] - G
    iters = np.zeros(N, dtype=np.int64)
    active = np.ones(N, dtype=bool)
    steps = n_iter if tol is None else max_iter

    def resid(vv):
        Gv = np.einsum("xpq,xq->xp", G, vv)
        lam = np.real(np.einsum("xp,xp->x", vv.conj(), Gv))
        return lam, np.linalg.norm(Gv - lam[:, None] * vv, axis=1)

    for _ in range(steps):
        if tol is not None:
            _, r = resid(v)
            active &= r > tol * bound
            if not active.any():
                break
        w = np.einsum("xpq,xq->xp", Gs[active], v[active])
        v[active] = w / np.linalg.norm(w, axis=1, keepdims=True)
        iters[active] += 1
    lam, r = resid(v)
    return v, lam, r, iters
