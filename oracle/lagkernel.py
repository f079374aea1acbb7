"""Lag kernel of the nullspace filters (oracle; test infrastructure).

Sec. IV-C: W = sum_r h_r h_r^H has Q x Q blocks W_qp with entries
[W_qp]_{st} = sum_r conj(h_r[n_t, p]) h_r[n_s, q] (Eq. 25).  Writing row s of
W_qp as a sequence w^s_qp[n_t] = [W_qp]_{st}, Eq. (26) gives

    [G(x)]_pq = sum_m ( sum_s w^s_qp[m + n_s] ) e^{-i 2 pi m.x}.

The inner sum is the lag kernel K_pq[m] computed here; m ranges over the
difference set Lambda - Lambda (m = n_t - n_s).  The filter vector index is
q|Lambda| + i (Eq. 14).
"""
from __future__ import annotations

import numpy as np

from .support import index_of


def gram_of_filters(h: np.ndarray) -> np.ndarray:
    """W = sum_r h_r h_r^H for filters stored as the columns of h."""
    h = np.asarray(h, dtype=np.complex128)
    return h @ h.conj().T


def lag_kernel(W: np.ndarray, lam: np.ndarray, lags: np.ndarray, Q: int) -> np.ndarray:
    """K[p, q, l] = sum over (s, t) with n_t - n_s = m_l of W[(q,s), (p,t)]."""
    L = len(lam)
    W4 = np.asarray(W).reshape(Q, L, Q, L)          # [q, s, p, t]
    idx = index_of(lags)
    K = np.zeros((Q, Q, len(lags)), dtype=np.complex128)
    # gather the (s, t) pairs of every lag once, then sum the W entries
    members = {}
    for s in range(L):
        for t in range(L):
            l = idx[tuple(int(v) for v in (lam[t] - lam[s]))]
            members.setdefault(l, []).append((s, t))
    for l, st in members.items():
        s_idx = np.array([a for a, _ in st])
        t_idx = np.array([b for _, b in st])
        # W4[q, s, p, t] summed over the listed (s, t), stored at [p, q]
        K[:, :, l] = W4[:, s_idx, :, t_idx].sum(axis=0).T
    return K


def lag_kernel_from_filters(h: np.ndarray, lam: np.ndarray, lags: np.ndarray,
                            Q: int) -> np.ndarray:
    """K from the filters via W (Eqs. 25-26)."""
    return lag_kernel(gram_of_filters(h), lam, lags, Q)
