"""Seeded synthetic multichannel MRI scans (the forward model only).

This module produces inputs for both the HIP path and the CPU oracle.  It
holds none of the estimation method's arithmetic: it draws a phantom, smooth
coil sensitivity maps and noisy Nyquist-sampled k-space following the signal
model of Eq. (1) of the paper (d_q(k) = FT{c_q rho}(k) + noise) and the
Fourier-series convention of Eqs. (2)-(4) (FOV [-1/2, 1/2)^D, unit k-space
spacing).

Grid convention (used everywhere in this repository): along a dimension of
length L, array index a corresponds to integer frequency k = a - floor(L/2)
and to position x = (a - floor(L/2)) / L.  Arrays are stored [z][y][x] with
the last dimension fastest; 2D arrays are [y][x].

Distributions (stated because the paper's data sets are not available; these
stand in for its brain and knee scans):
  * phantom: E ellipses (2D) or ellipsoids (3D); centre ~ U[-0.3, 0.3]^D,
    semi-axes ~ U[0.05, 0.25], uniform rotation, complex intensity
    U[0.3, 1] * exp(i U[0, 2 pi)); a shape is redrawn until it lies inside
    ||x||_inf <= 0.45, so the object has background around it;
  * maps: three Gaussian bumps per coil with centres on a ring (2D) or a
    Fibonacci sphere (3D) of radius U[0.55, 0.75], widths U[0.25, 0.5],
    complex amplitudes U[0.5, 1] * exp(i U[0, 2 pi)); then normalised to unit
    root-sum-of-squares at every voxel;
  * k-space: centred orthonormal DFT of rho * c_q plus circular complex
    Gaussian noise with variance sigma^2 = mean_{q,x} |rho c_q|^2 / 10^(SNR/10)
    (sigma^2 / 2 per real component) on every sample.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Scan:
    """One synthetic scan.  All arrays are complex128 unless noted."""

    grid: tuple            # image grid (Nz, Ny, Nx) or (Ny, Nx)
    Q: int
    acs_shape: tuple       # ACS block shape, same rank as grid
    image: np.ndarray      # rho(x) on the grid
    maps: np.ndarray       # [Q, *grid] true maps, unit RSS
    kspace: Optional[np.ndarray]  # [Q, *grid] noisy k-space (None if not kept)
    acs: np.ndarray        # [Q, *acs_shape] noisy centred ACS block
    sigma2: float          # noise variance per complex sample
    seed: int


def grid_positions(n: int) -> np.ndarray:
    """Positions x_a = (a - floor(n/2)) / n of a centred grid of length n."""
    return (np.arange(n) - n // 2) / float(n)


def centred_fft(x: np.ndarray, axes: Sequence[int]) -> np.ndarray:
    """Orthonormal DFT with e^{-i 2 pi k x}, centred index convention."""
    return np.fft.fftshift(
        np.fft.fftn(np.fft.ifftshift(x, axes=axes), axes=axes, norm="ortho"),
        axes=axes)


def centred_ifft(x: np.ndarray, axes: Sequence[int]) -> np.ndarray:
    """Inverse of centred_fft (e^{+i 2 pi k x})."""
    return np.fft.fftshift(
        np.fft.ifftn(np.fft.ifftshift(x, axes=axes), axes=axes, norm="ortho"),
        axes=axes)


def _random_rotation(rng: np.random.Generator, D: int) -> np.ndarray:
    if D == 2:
        th = rng.uniform(0.0, np.pi)
        c, s = np.cos(th), np.sin(th)
        return np.array([[c, -s], [s, c]])
    a = rng.standard_normal((3, 3))
    q, r = np.linalg.qr(a)
    q = q * np.sign(np.diag(r))[None, :]
    return q


def _draw_shapes(rng: np.random.Generator, D: int, E: int):
    shapes = []
    while len(shapes) < E:
        centre = rng.uniform(-0.3, 0.3, size=D)
        axes = rng.uniform(0.05, 0.25, size=D)
        rot = _random_rotation(rng, D)
        amp = rng.uniform(0.3, 1.0) * np.exp(1j * rng.uniform(0.0, 2 * np.pi))
        # half extent of the rotated ellipsoid along each coordinate axis
        half = np.sqrt(((rot * axes[None, :]) ** 2).sum(axis=1))
        if np.all(np.abs(centre) + half <= 0.45):
            shapes.append((centre, axes, rot, amp))
    return shapes


def _coords(grid: Sequence[int]) -> list:
    """Broadcastable coordinate arrays, one per dimension (slowest first)."""
    D = len(grid)
    out = []
    for d, n in enumerate(grid):
        shape = [1] * D
        shape[d] = n
        out.append(grid_positions(n).reshape(shape))
    return out


def _phantom(grid, shapes) -> np.ndarray:
    xs = _coords(grid)
    img = np.zeros(tuple(grid), dtype=np.complex128)
    for centre, axes, rot, amp in shapes:
        # coordinates in the ellipsoid frame: u = rot^T (x - centre)
        rel = [x - c for x, c in zip(xs, centre)]
        inside = np.zeros(tuple(grid), dtype=np.float64)
        for j in range(len(grid)):
            u = sum(rot[d, j] * rel[d] for d in range(len(grid)))
            inside = inside + (u / axes[j]) ** 2
        img = img + amp * (inside <= 1.0)
    return img


def _fibonacci_dirs(Q: int) -> np.ndarray:
    i = np.arange(Q) + 0.5
    phi = np.arccos(1 - 2 * i / Q)
    theta = np.pi * (1 + 5 ** 0.5) * i
    return np.stack([np.cos(phi), np.sin(phi) * np.sin(theta),
                     np.sin(phi) * np.cos(theta)], axis=1)


def _draw_bumps(rng: np.random.Generator, D: int, Q: int) -> list:
    """Three Gaussian bumps per coil: [(centre, width, amplitude)] per q."""
    dirs3 = _fibonacci_dirs(Q) if D == 3 else None
    bumps = []
    for q in range(Q):
        coil = []
        for _ in range(3):
            radius = rng.uniform(0.55, 0.75)
            if D == 2:
                ang = 2 * np.pi * q / Q + rng.uniform(-0.2, 0.2)
                centre = radius * np.array([np.sin(ang), np.cos(ang)])
            else:
                d = dirs3[q] + rng.uniform(-0.2, 0.2, size=3)
                centre = radius * d / np.linalg.norm(d)
            width = rng.uniform(0.25, 0.5)
            amp = rng.uniform(0.5, 1.0) * np.exp(1j * rng.uniform(0, 2 * np.pi))
            coil.append((centre, width, amp))
        bumps.append(coil)
    return bumps


def _raw_map(xs, coil_bumps) -> np.ndarray:
    """One coil's bump mixture before the RSS normalisation."""
    out = 0.0
    for centre, width, amp in coil_bumps:
        r2 = sum((x - c) ** 2 for x, c in zip(xs, centre))
        out = out + amp * np.exp(-r2 / (2 * width ** 2))
    return out


def _maps(rng: np.random.Generator, grid, Q: int) -> np.ndarray:
    xs = _coords(grid)
    bumps = _draw_bumps(rng, len(grid), Q)
    maps = np.zeros((Q,) + tuple(grid), dtype=np.complex128)
    for q in range(Q):
        maps[q] = maps[q] + _raw_map(xs, bumps[q])
    rss = np.sqrt((np.abs(maps) ** 2).sum(axis=0))
    return maps / rss[None]


def centre_block(arr: np.ndarray, shape: Sequence[int]) -> np.ndarray:
    """Centred block of the trailing dimensions of arr (index a <-> k)."""
    sl = [slice(None)] * (arr.ndim - len(shape))
    for n, a in zip(arr.shape[-len(shape):], shape):
        lo = n // 2 - a // 2
        sl.append(slice(lo, lo + a))
    return arr[tuple(sl)]


def make_scan(seed: int, grid: Sequence[int], Q: int, acs_shape: Sequence[int],
              n_shapes: int, snr_db: float, keep_kspace: bool = True) -> Scan:
    """Draw one scan.  Deterministic for a given seed and arguments."""
    grid = tuple(int(g) for g in grid)
    acs_shape = tuple(int(a) for a in acs_shape)
    D = len(grid)
    if len(acs_shape) != D or D not in (2, 3):
        raise ValueError("grid and acs_shape must both have rank 2 or 3")
    rng = np.random.Generator(np.random.PCG64(seed))
    shapes = _draw_shapes(rng, D, n_shapes)
    image = _phantom(grid, shapes)
    maps = _maps(rng, grid, Q)
    axes = tuple(range(1, D + 1))
    coil = maps * image[None]
    ksp = centred_fft(coil, axes)
    sigma2 = float(np.mean(np.abs(coil) ** 2) / 10 ** (snr_db / 10.0))
    noise = (rng.standard_normal(ksp.shape) + 1j * rng.standard_normal(ksp.shape))
    ksp = ksp + np.sqrt(sigma2 / 2.0) * noise
    acs = np.ascontiguousarray(centre_block(ksp, acs_shape))
    return Scan(grid=grid, Q=Q, acs_shape=acs_shape, image=image, maps=maps,
                kspace=ksp if keep_kspace else None, acs=acs, sigma2=sigma2,
                seed=seed)


def as_device_input(acs: np.ndarray) -> np.ndarray:
    """The ACS as the GPU receives it: complex64.  The oracle is run on this
    same rounded array (widened back to complex128) so both sides see
    identical inputs."""
    return np.ascontiguousarray(acs.astype(np.complex64))


def _acs_dft(n: int, a: int) -> np.ndarray:
    """[a, n] rows of the centred orthonormal DFT for the a central
    frequencies k = -floor(a/2) ... (e^{-i 2 pi k x})."""
    k = np.arange(a) - a // 2
    return np.exp(-2j * np.pi * np.outer(k, grid_positions(n))) / np.sqrt(n)


def make_acs_scan(seed: int, grid: Sequence[int], Q: int, acs_shape: Sequence[int],
                  n_shapes: int, snr_db: float) -> Scan:
    """Draw a scan too large to hold as full k-space: only the ACS block.

    Same phantom and map distributions as make_scan.  Each coil image
    rho * c_q is formed in turn and its centred ACS block taken by a
    separable partial DFT (exact: the same samples the full orthonormal DFT
    would give).  The noise variance comes from the mean coil energy over
    the whole grid as in make_scan; noise is drawn for the ACS samples only
    (independent per sample, so its statistics there are those of the full
    k-space).  image, maps and kspace are not kept (maps is None-shaped: an
    empty array)."""
    grid = tuple(int(g) for g in grid)
    acs_shape = tuple(int(a) for a in acs_shape)
    D = len(grid)
    if len(acs_shape) != D or D not in (2, 3):
        raise ValueError("grid and acs_shape must both have rank 2 or 3")
    rng = np.random.Generator(np.random.PCG64(seed))
    shapes = _draw_shapes(rng, D, n_shapes)
    image = _phantom(grid, shapes)
    xs = _coords(grid)
    bumps = _draw_bumps(rng, D, Q)
    rss2 = np.zeros(grid, dtype=np.float64)
    for q in range(Q):
        rss2 += np.abs(_raw_map(xs, bumps[q])) ** 2
    inv_rss = 1.0 / np.sqrt(rss2)
    del rss2
    mats = [_acs_dft(n, a) for n, a in zip(grid, acs_shape)]
    acs = np.empty((Q,) + acs_shape, dtype=np.complex128)
    energy = 0.0
    for q in range(Q):
        coil = _raw_map(xs, bumps[q]) * inv_rss * image
        energy += float(np.sum(np.abs(coil) ** 2))
        blk = coil
        for d in range(D - 1, -1, -1):
            blk = np.moveaxis(np.tensordot(mats[d], blk, axes=([1], [d])), 0, d)
        acs[q] = blk
    sigma2 = energy / (Q * float(np.prod(grid))) / 10 ** (snr_db / 10.0)
    noise = rng.standard_normal(acs.shape) + 1j * rng.standard_normal(acs.shape)
    acs = acs + np.sqrt(sigma2 / 2.0) * noise
    return Scan(grid=grid, Q=Q, acs_shape=acs_shape, image=np.empty(0),
                maps=np.empty(0), kspace=None, acs=np.ascontiguousarray(acs),
                sigma2=sigma2, seed=seed)
