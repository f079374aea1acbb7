"""Many small partial SVDs (oracle; test infrastructure).

Sec. I and Sec. V note that the batched small eigen-problems the method
accelerates also serve locally low-rank models: each patch's Casorati
matrix (rows: the patch's pixels; columns: channels or frames) is replaced
by its best rank-r approximation.  The oracle takes numpy's SVD of each
matrix: the r largest singular values, the right singular vectors and the
truncated reconstruction U_r diag(sigma_r) V_r^H (Eckart-Young).
"""
from __future__ import annotations

import numpy as np


def partial_svd(X: np.ndarray, r: int):
    """X: [B, Q, m] (column q of patch b is X[b, q]); the matrix of patch b
    is M_b = X[b].T (m x Q).  Returns (sigma [B, r] descending,
    V [B, Q, r] right singular vectors, Xr [B, Q, m] the rank-r part in the
    same layout)."""
    M = np.transpose(np.asarray(X, dtype=np.complex128), (0, 2, 1))   # [B, m, Q]
    U, s, Vh = np.linalg.svd(M, full_matrices=False)
    Mr = np.einsum("bik,bk,bkq->biq", U[:, :, :r], s[:, :r], Vh[:, :r, :])
    V = np.conj(np.transpose(Vh[:, :r, :], (0, 2, 1)))
    return s[:, :r], V, np.transpose(Mr, (0, 2, 1))
