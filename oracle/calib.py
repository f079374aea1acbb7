"""Calibration matrix C and its Gram C^H C (oracle; test infrastructure).

Conventions.  The ACS array s[q][a_0]...[a_{D-1}] holds the Nyquist samples
s_q[k] with k_d = a_d - floor(A_d / 2) (Eqs. 2-4).  Following Eq. (5), row n of
the block C_q holds (s_q[n - m])_{m in Lambda}, so (C h)[n] is the annihilation
sum of Eq. (5), and C = [C_1 ... C_Q] (Eq. 14) has column index q|Lambda| + i.

Sec. IV-A: with masking neglected, column i of C_p^H C_q is a shift of the
single correlation (s_q * s_p^*[-.]), so

    (C_p^H C_q)_{ij} = R_pq[n_i - n_j],   R_pq[d] = sum_k conj(s_p[k]) s_q[k+d]

with samples outside the ACS taken as zero.  That is exactly C_full^H C_full
where C_full keeps every row n for which some s_q[n - m] is inside the ACS.
The oracle computes R_pq by direct summation (no FFT).
"""
from __future__ import annotations

import itertools

import numpy as np

from .support import index_of


def _overlap(A: tuple, d: tuple):
    """Index slices (for k and for k + d) of the overlap of the ACS with its
    shift by d."""
    src, dst = [], []
    for n, dd in zip(A, d):
        lo = max(0, -dd)
        hi = min(n, n - dd)
        if hi <= lo:
            return None
        src.append(slice(lo, hi))
        dst.append(slice(lo + dd, hi + dd))
    return tuple(src), tuple(dst)


def correlation_lags(acs: np.ndarray, lags: np.ndarray) -> np.ndarray:
    """R[p, q, l] = sum_k conj(s_p[k]) s_q[k + d_l] by direct summation.

    acs: [Q, *A] complex; lags: [L, D] integer offsets.  Returns complex128
    [Q, Q, L]."""
    acs = np.asarray(acs, dtype=np.complex128)
    Q = acs.shape[0]
    A = acs.shape[1:]
    R = np.zeros((Q, Q, len(lags)), dtype=np.complex128)
    for l, d in enumerate(lags):
        ov = _overlap(A, tuple(int(v) for v in d))
        if ov is None:
            continue
        src, dst = ov
        x = acs[(slice(None),) + src].reshape(Q, -1)   # s_p[k]
        y = acs[(slice(None),) + dst].reshape(Q, -1)   # s_q[k + d]
        R[:, :, l] = np.conj(x) @ y.T
    return R


def gram_from_lags(R: np.ndarray, lam: np.ndarray, lags: np.ndarray) -> np.ndarray:
    """Gram[(p,i),(q,j)] = R_pq[n_i - n_j]; index q|Lambda| + i (Eq. 14)."""
    Q = R.shape[0]
    L = len(lam)
    idx = index_of(lags)
    lag_of = np.array([[idx[tuple(int(v) for v in (lam[i] - lam[j]))]
                        for j in range(L)] for i in range(L)])
    G = R[:, :, lag_of]                      # [p, q, i, j]
    return G.transpose(0, 2, 1, 3).reshape(Q * L, Q * L)


def calibration_matrix(acs: np.ndarray, lam: np.ndarray,
                       rows: str = "full") -> np.ndarray:
    """Explicit C (Eq. 14) with C_q[n, i] = s_q[n - n_i].

    rows="full": every n of the box spanned by ACS + Lambda (rows that are all
    zero do not change C^H C); rows="valid": only n with n - Lambda inside the
    ACS (no implicit zeros)."""
    acs = np.asarray(acs, dtype=np.complex128)
    Q = acs.shape[0]
    A = acs.shape[1:]
    D = len(A)
    lo_k = [-(a // 2) for a in A]
    hi_k = [a - 1 - a // 2 for a in A]
    mn = lam.min(axis=0)
    mx = lam.max(axis=0)
    ranges = [range(lo_k[d] + int(mn[d]), hi_k[d] + int(mx[d]) + 1)
              for d in range(D)]
    row_list = []
    for n in itertools.product(*ranges):
        ks = [tuple(n[d] - int(m[d]) for d in range(D)) for m in lam]
        inside = [all(lo_k[d] <= k[d] <= hi_k[d] for d in range(D)) for k in ks]
        if rows == "valid" and not all(inside):
            continue
        row = np.zeros(Q * len(lam), dtype=np.complex128)
        for i, (k, ok) in enumerate(zip(ks, inside)):
            if ok:
                a = tuple(k[d] - lo_k[d] for d in range(D))
                row[np.arange(Q) * len(lam) + i] = acs[(slice(None),) + a]
        row_list.append(row)
    return np.array(row_list).reshape(-1, Q * len(lam))
