"""The oracle's steps chained end to end (test infrastructure).

Follows the naive nullspace algorithm of Sec. III-D with the PISCO choices
of Sec. IV: ellipsoidal support (IV-B), the correlation form of C^H C (IV-A),
G(x) from the lag sums of W (IV-C), a low-resolution estimation grid with
sinc interpolation (IV-D) and power iteration (IV-E).  Every intermediate is
returned so that each stage of the HIP path can be compared with it.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from . import calib, eig, gx, lagkernel, maps, nullspace, support


@dataclasses.dataclass
class Result:
    lam: np.ndarray
    lags: np.ndarray
    R: np.ndarray
    gram: np.ndarray
    split: nullspace.Split
    K: np.ndarray                 # lag kernel of the NULL filters (Eq. 26)
    G: np.ndarray                 # [N_lr, Q, Q]
    c_lr: np.ndarray              # [Q, *grid_lr] after power iteration
    lam_min: np.ndarray           # [N_lr]
    iters: np.ndarray
    rho_lr: np.ndarray            # apodized low-res images [Q, *grid_lr]
    c_ref: np.ndarray             # after the phase reference
    maps: Optional[np.ndarray]    # [Q, *grid_out], unit RSS


def estimate(acs: np.ndarray, radius: float, grid_lr, grid_out=None,
             thresh: float = 0.05, n_iter: int = 10, tol: float | None = None,
             phase: str = "combined", shape: str = "ellipsoid",
             rows: str = "full") -> Result:
    """rows="full": the correlation Gram of Sec. IV-A (masking neglected,
    = C_full^H C_full); rows="valid": C_valid^H C_valid from the explicit
    rows of C with no implicit zeros (the masked form)."""
    acs = np.asarray(acs, dtype=np.complex128)
    Q = acs.shape[0]
    D = acs.ndim - 1
    lam = support.kernel_support(D, radius, shape)
    lags = support.difference_set(lam)
    R = calib.correlation_lags(acs, lags)
    if rows == "valid":
        C = calib.calibration_matrix(acs, lam, rows="valid")
        gram = C.conj().T @ C
    else:
        gram = calib.gram_from_lags(R, lam, lags)
    sp = nullspace.split_from_gram(gram, thresh)
    K = lagkernel.lag_kernel_from_filters(sp.null, lam, lags, Q)
    x = gx.grid_points(grid_lr)
    G = gx.gx_from_lag_kernel(K, lags, x)
    G = 0.5 * (G + np.conj(np.transpose(G, (0, 2, 1))))
    c, lmin, _, iters = eig.power_iteration(G, float(len(lam)), n_iter, tol)
    c_lr = c.T.reshape((Q,) + tuple(grid_lr))
    rho = maps.apodized_lowres(acs, grid_lr)
    if phase == "combined":
        c_ref, _ = maps.phase_reference(c_lr, rho)
    else:
        c_ref = maps.coil_reference(c_lr)
    out = None
    if grid_out is not None:
        out = maps.normalize_rss(maps.interpolate(c_ref, grid_out))
    return Result(lam, lags, R, gram, sp, K, G, c_lr, lmin, iters, rho, c_ref, out)
