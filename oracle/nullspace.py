"""Approximate nullspace of C (oracle; test infrastructure).

Sec. III-A: the filters h_r are the approximate nullspace vectors of C,
found with the SVD.  Sec. III-B footnote: with singular values sorted from
largest to smallest, the n-th right singular vector is null when
sigma_n < 0.05 sigma_1.  Sec. IV-A: C and C^H C share that structure, so the
oracle takes the eigen-decomposition of the Gram: its eigenvalues are
lambda_n = sigma_n^2 and the rule reads lambda_n < 0.05^2 lambda_1.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Split:
    eigvals: np.ndarray     # [n] descending, clipped at 0
    vectors: np.ndarray     # [n, n] column k belongs to eigvals[k]
    r_signal: int           # number of eigenvalues kept as signal
    r_null: int             # R, the nullspace dimension
    gap: float              # relative distance of the spectrum from the threshold

    @property
    def signal(self) -> np.ndarray:
        return self.vectors[:, : self.r_signal]

    @property
    def null(self) -> np.ndarray:
        return self.vectors[:, self.r_signal:]


def split_from_gram(gram: np.ndarray, thresh: float = 0.05) -> Split:
    """Eigen-decomposition of the Hermitian Gram and the sigma rule."""
    gram = np.asarray(gram, dtype=np.complex128)
    gram = 0.5 * (gram + gram.conj().T)
    w, V = np.linalg.eigh(gram)
    w = w[::-1].copy()
    V = V[:, ::-1].copy()
    w = np.maximum(w, 0.0)
    level = thresh * thresh * w[0]
    null = w < level
    r_s = int(np.count_nonzero(~null))
    # signal eigenvalues come first because the spectrum is sorted
    gap = np.inf
    if r_s > 0 and level > 0:
        gap = min(gap, w[r_s - 1] / level - 1.0)
    if r_s < len(w) and level > 0:
        gap = min(gap, 1.0 - w[r_s] / level)
    return Split(w, V, r_s, len(w) - r_s, float(gap))


def split_from_svd(C: np.ndarray, thresh: float = 0.05):
    """The same split taken from the SVD of an explicit C (Sec. III-A).

    Returns (singular values, right singular vectors as columns, r_signal);
    right singular vectors past min(P, n) are null by construction."""
    C = np.asarray(C, dtype=np.complex128)
    n = C.shape[1]
    _, s, Vh = np.linalg.svd(C, full_matrices=True)
    sig = np.zeros(n)
    sig[: len(s)] = s
    r_s = int(np.count_nonzero(sig >= thresh * sig[0]))
    return sig, Vh.conj().T, r_s


def projector(V: np.ndarray) -> np.ndarray:
    """Orthogonal projector V V^H onto the span of orthonormal columns V."""
    return V @ V.conj().T
