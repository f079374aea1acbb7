"""Writes tests/golden/app3d_reference.npz: sampled FP64 oracle results for
the 3D application workload (256 x 256 x 128 grid, 32 channels, 32^3 ACS,
radius 5, n = 16480, maps estimated on 56^3 and interpolated).

The whole problem is too large for the oracle to run inside a test, so this
script runs it once, calling only oracle/ (and synth/ for the seeded input),
and stores what the GPU test compares at sampled points:
  * the leading Gram eigenvalues and the signal rank (Sec. III-B rule);
  * G(x) (packed upper triangle) at 256 sampled low-res voxels (Eq. 26);
  * lambda_min by 10 power-iteration steps from e_q* (Sec. IV-E) and by the
    exact per-voxel eigen-decomposition, with the eigen-gap, at 16384
    sampled low-res voxels;
  * the final maps (power iteration, phase reference of Sec. IV-D,
    periodic sinc interpolation, unit RSS) and the maps from the exact
    per-voxel eigenvectors through the same steps, at 4096 sampled output
    voxels, with the mask of voxels where the map is defined (coil-combined
    apodized image |m| >= 1e-3 max|m|, eroded by one low-res voxel).

Run from the repository root:  python tests/golden/make_app3d_reference.py
(about 40 minutes and 30 GB of host memory on 8 cores).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import calib, eig, gx, lagkernel, maps, nullspace, support  # noqa: E402
from synth import as_device_input, workloads  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "app3d_reference.npz")


def log(msg, t0=[time.time()]):
    print(f"[{time.time() - t0[0]:7.1f} s] {msg}", flush=True)


def lowres_mask(c_lr, rho):
    from scipy.ndimage import binary_erosion
    m = np.abs(np.sum(np.conj(c_lr) * rho, axis=0))
    return binary_erosion(m >= 1e-3 * m.max(), iterations=1)


def nearest_lowres(idx_out, grid_out, grid_lr):
    """Low-res voxel nearest to each sampled output voxel (flat indices)."""
    coords = np.unravel_index(idx_out, grid_out)
    near = []
    for c, n_out, n_lr in zip(coords, grid_out, grid_lr):
        x = (c - n_out // 2) / n_out
        near.append(np.round(x * n_lr + n_lr // 2).astype(int) % n_lr)
    return np.ravel_multi_index(near, grid_lr)


def main():
    w = workloads.APP_3D
    Q, grid, grid_lr = w.Q, tuple(w.grid), tuple(w.grid_lr)
    acs = as_device_input(w.scan().acs).astype(np.complex128)
    log("ACS drawn")
    lam = support.kernel_support(3, w.radius)
    lags = support.difference_set(lam)
    L = len(lam)
    R = calib.correlation_lags(acs, lags)
    log(f"correlation lags ({len(lags)})")
    gram = calib.gram_from_lags(R, lam, lags)
    del R
    log(f"Gram {gram.shape}")
    sp = nullspace.split_from_gram(gram, 0.05)
    del gram
    log(f"split: r_signal {sp.r_signal}, gap {sp.gap:.3e}")
    eigvals = sp.eigvals[: sp.r_signal + 64].copy()
    K = lagkernel.lag_kernel_from_filters(sp.null, lam, lags, Q)
    r_signal, gap = sp.r_signal, sp.gap
    del sp
    log("lag kernel")
    x = gx.grid_points(grid_lr)
    G = gx.gx_from_lag_kernel(K, lags, x)
    G = 0.5 * (G + np.conj(np.transpose(G, (0, 2, 1))))
    del K
    log("G(x)")
    rng = np.random.default_rng(20000)
    N_lr = len(x)
    idx_g = np.sort(rng.choice(N_lr, 256, replace=False))
    idx_lam = np.sort(rng.choice(N_lr, 16384, replace=False))
    iu = np.triu_indices(Q)
    G_sample = np.ascontiguousarray(G[idx_g][:, iu[0], iu[1]].T.astype(np.complex64))
    c, lmin, _, _ = eig.power_iteration(G, float(L), 10)
    log("power iteration")
    lam_ex, c_ex, lam2 = eig.smallest_exact(G)
    del G
    log("exact per-voxel eigenvectors")
    rho = maps.apodized_lowres(acs, grid_lr)
    c_lr = np.ascontiguousarray(c.T.reshape((Q,) + grid_lr))
    cx_lr = np.ascontiguousarray(c_ex.T.reshape((Q,) + grid_lr))
    del c, c_ex
    mask_lr = lowres_mask(c_lr, rho)
    N_out = int(np.prod(grid))
    idx_out = np.sort(rng.choice(N_out, 4096, replace=False))
    near = nearest_lowres(idx_out, grid, grid_lr)
    out = {}
    for tag, cl in (("maps", c_lr), ("maps_exact", cx_lr)):
        cref, _ = maps.phase_reference(cl, rho)
        m = maps.normalize_rss(maps.interpolate(cref, grid)).reshape(Q, -1)
        out[tag] = np.ascontiguousarray(m[:, idx_out].astype(np.complex64))
        del m, cref
        log(tag)
    np.savez(OUT, workload=np.array(w.name), seed=np.array(w.seeds[0]),
             r_signal=np.array(r_signal), gap=np.array(gap), eigvals=eigvals,
             idx_g=idx_g, G_sample=G_sample, idx_lam=idx_lam,
             lam_min=lmin[idx_lam], lam_exact=lam_ex[idx_lam], lam_2=lam2[idx_lam],
             idx_out=idx_out, mask_out=mask_lr.reshape(-1)[near],
             maps=out["maps"], maps_exact=out["maps_exact"])
    log(f"wrote {OUT}")


if __name__ == "__main__":
    main()
