"""Phase reference, interpolation and normalisation (oracle; test infrastructure).

Sec. IV-D: maps are estimated on a low-resolution grid and brought to the
output grid by periodic sinc interpolation (zero-padded FFT).  Before that,
a scaling alpha(x) (Sec. II) fixes the otherwise arbitrary per-voxel phase:
the current map estimates coil-combine a Gaussian-apodized low-resolution
Fourier reconstruction of the calibration data and alpha(x) cancels the phase
of that combination.  Sec. V: magnitudes are normalised by sum of squares;
phase referenced to one coil is the alternative rule.

Readings of points the paper leaves open (this repository's choices):
  * apodization g[k] = prod_d exp(-k_d^2 / (2 (A_d/4)^2));
  * coil combination m(x) = sum_q conj(c_q(x)) rho~_q(x) with unit-norm c;
  * alpha(x) = m(x)/|m(x)| where |m(x)| > 1e-12 max|m|, else 1;
  * interpolation: centred DFT of the low-res samples, the band
    k in [-floor(N/2), ceil(N/2) - 1] kept and, for even N upsampled to a
    larger grid, the k = -N/2 coefficient split half/half onto +-N/2;
  * unit root-sum-of-squares after interpolation; zero stays zero.
"""
from __future__ import annotations

import numpy as np


def _positions(n: int) -> np.ndarray:
    return (np.arange(n) - n // 2) / float(n)


def apodized_lowres(acs: np.ndarray, grid_lr) -> np.ndarray:
    """rho~_q(x) = sum_{k in ACS} g[k] s_q[k] e^{+i 2 pi k.x} on grid_lr.

    Separable direct evaluation, one dimension at a time; [Q, *grid_lr]."""
    out = np.asarray(acs, dtype=np.complex128)
    A = out.shape[1:]
    for d, (a, n) in enumerate(zip(A, grid_lr)):
        k = np.arange(a) - a // 2
        g = np.exp(-(k.astype(np.float64) ** 2) / (2.0 * (a / 4.0) ** 2))
        E = np.exp(2j * np.pi * np.outer(_positions(n), k)) * g[None, :]   # [n, a]
        out = np.moveaxis(np.tensordot(E, out, axes=([1], [d + 1])), 0, d + 1)
    return out


def phase_reference(c: np.ndarray, rho: np.ndarray, rel_floor: float = 1e-12):
    """c <- c * m/|m| with m = sum_q conj(c_q) rho~_q.  c, rho: [Q, *grid]."""
    m = np.sum(np.conj(c) * rho, axis=0)
    mag = np.abs(m)
    ok = mag > rel_floor * mag.max() if mag.size else mag > 0
    alpha = np.ones_like(m)
    alpha[ok] = m[ok] / mag[ok]
    return c * alpha[None], alpha


def coil_reference(c: np.ndarray, q_ref: int = 0) -> np.ndarray:
    """Alternative rule of Sec. V: c <- c * conj(c_ref)/|c_ref|."""
    ref = c[q_ref]
    mag = np.abs(ref)
    alpha = np.ones_like(ref)
    ok = mag > 0
    alpha[ok] = np.conj(ref[ok]) / mag[ok]
    return c * alpha[None]


def sinc_matrix(n_in: int, n_out: int) -> np.ndarray:
    """[n_out, n_in] periodic sinc interpolation from n_in centred samples."""
    if n_out < n_in:
        raise ValueError("interpolation only upsamples")
    x = _positions(n_in)
    y = _positions(n_out)
    ks = list(range(-(n_in // 2), (n_in + 1) // 2))
    w = [1.0] * len(ks)
    if n_in % 2 == 0 and n_out > n_in:
        w[0] = 0.5
        ks.append(n_in // 2)
        w.append(0.5)
    ks = np.array(ks, dtype=np.float64)
    w = np.array(w)
    fwd = np.exp(-2j * np.pi * np.outer(ks, x)) / n_in        # [K, n_in]
    inv = np.exp(2j * np.pi * np.outer(y, ks)) * w[None, :]   # [n_out, K]
    return inv @ fwd


def interpolate(c_lr: np.ndarray, grid_out) -> np.ndarray:
    """Separable periodic sinc interpolation of [Q, *grid_lr] to grid_out."""
    out = np.asarray(c_lr, dtype=np.complex128)
    for d, n in enumerate(grid_out):
        T = sinc_matrix(out.shape[d + 1], n)
        out = np.moveaxis(np.tensordot(T, out, axes=([1], [d + 1])), 0, d + 1)
    return out


def normalize_rss(c: np.ndarray) -> np.ndarray:
    """c(x) / ||c(x)||_2 over coils; voxels with zero norm stay zero."""
    rss = np.sqrt(np.sum(np.abs(c) ** 2, axis=0))
    out = np.zeros_like(c)
    ok = rss > 0
    out[:, ok] = c[:, ok] / rss[ok]
    return out


def support_mask(lam_min_lr: np.ndarray, bound: float, grid_out,
                 thresh: float = 0.1) -> np.ndarray:
    """Binary mask of the image support (Sec. III-D, optional last step).

    The smallest singular value of H(x) is about zero inside the support and
    clearly positive outside it (Sec. III-B, III-C).  Its square is
    lambda_min(G(x)); normalised by |Lambda| (the scale the paper plots) the
    map lies in [0, 1].  Reading taken here: the low-resolution map
    lambda_min / |Lambda| is brought to the output grid by the same periodic
    sinc interpolation as the maps, and a voxel is inside the support where
    the interpolated value is below `thresh`.  Returns a bool array shaped
    grid_out."""
    lr = np.asarray(lam_min_lr, dtype=np.float64) / float(bound)
    up = interpolate(lr[None].astype(np.complex128), grid_out)[0]
    return up.real < thresh
