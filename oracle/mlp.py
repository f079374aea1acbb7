"""Learned warm start for the per-voxel power iteration (oracle; test
infrastructure only, never called by the product path).

Not in the paper.  The power iteration of Sec. IV-E starts every voxel from
a fixed vector; here a small network predicts a start vector close to the
eigenvector of G(x) for its smallest eigenvalue, so that fewer steps reach a
given residual.  The definitions below are the reference for the GPU
kernels; everything is FP64 numpy.

Network (this repository's reading of the design):
  features z(x) = [ G_qq(x) / |Lambda|                       (Q reals),
                    Re, Im of G_pq(x) / |Lambda| for p < q      (Q(Q-1) reals),
                    Re, Im of the neighbour vector n(x)          (2Q reals) ]
  h1 = relu(W1 z + b1),  h2 = relu(W2 h1 + b2),  y = W3 h2 + b3   (2Q reals)
  c_hat = n + (y_re + i y_im)                      (a correction of n)
The neighbour vector n(x) is the eigenvector found (from the plain start) at
the parent voxel of a grid coarser by two per dimension, with its largest-
magnitude entry rotated to be real and positive.

Loss per voxel (gauge invariant: any e^{i phi} c_hat scores the same):
  L = 1 - |c_hat^H c|^2 / ||c_hat||^2,  c the unit target eigenvector,
averaged over the batch.  The parameters are the flat vector
  theta = [W1 (H x Din, row-major), b1, W2 (H x H), b2, W3 (2Q x H), b3].
"""
from __future__ import annotations

import numpy as np

HIDDEN = 256


def dims(Q: int, hidden: int = HIDDEN):
    """(Din, H, Dout)."""
    return Q * Q + 2 * Q, hidden, 2 * Q


def param_count(Q: int, hidden: int = HIDDEN) -> int:
    din, h, dout = dims(Q, hidden)
    return h * din + h + h * h + h + dout * h + dout


def unpack(theta: np.ndarray, Q: int, hidden: int = HIDDEN):
    din, h, dout = dims(Q, hidden)
    o = 0
    out = []
    for shape in ((h, din), (h,), (h, h), (h,), (dout, h), (dout,)):
        size = int(np.prod(shape))
        out.append(theta[o:o + size].reshape(shape))
        o += size
    return out


def gauge_fix(v: np.ndarray) -> np.ndarray:
    """Rotate each vector (rows of v, [N, Q]) so that its largest-magnitude
    entry (lowest index on ties) is real and positive; zero rows stay zero."""
    v = np.asarray(v, dtype=np.complex128)
    k = np.argmax(np.abs(v), axis=1)
    a = v[np.arange(len(v)), k]
    mag = np.abs(a)
    ph = np.where(mag > 0, np.conj(a) / np.where(mag > 0, mag, 1.0), 1.0)
    return v * ph[:, None]


def features(G: np.ndarray, nb: np.ndarray, bound: float) -> np.ndarray:
    """z(x) for G [N, Q, Q] (Hermitian) and neighbour vectors nb [N, Q]."""
    G = np.asarray(G, dtype=np.complex128)
    N, Q, _ = G.shape
    iu = np.triu_indices(Q, 1)
    diag = np.real(np.einsum("xqq->xq", G)) / bound
    off = G[:, iu[0], iu[1]] / bound
    offr = np.stack([off.real, off.imag], axis=2).reshape(N, -1)
    nbr = np.stack([nb.real, nb.imag], axis=2).reshape(N, -1)
    return np.concatenate([diag, offr, nbr], axis=1)


def forward(theta, z, nb, Q: int, hidden: int = HIDDEN):
    """Returns (c_hat [N, Q] complex, cache for backward)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, Q, hidden)
    a1 = z @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    y = h2 @ W3.T + b3
    c_hat = nb + (y[:, 0::2] + 1j * y[:, 1::2])
    return c_hat, (z, a1, h1, a2, h2)


def loss(c_hat: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Per-voxel loss 1 - |c_hat^H c|^2 / ||c_hat||^2 (c unit)."""
    s = np.sum(np.conj(c_hat) * c, axis=1)
    n = np.sum(np.abs(c_hat) ** 2, axis=1)
    return 1.0 - np.abs(s) ** 2 / n


def loss_grad(c_hat: np.ndarray, c: np.ndarray) -> np.ndarray:
    """d L / d(Re c_hat) + i d L / d(Im c_hat) per voxel, from differentiating
    |s|^2 / n with s = c_hat^H c and n = ||c_hat||^2:
      g = -(2 / n) (conj(s) c - (|s|^2 / n) c_hat)."""
    s = np.sum(np.conj(c_hat) * c, axis=1)
    n = np.sum(np.abs(c_hat) ** 2, axis=1)
    return -(2.0 / n)[:, None] * (np.conj(s)[:, None] * c
                                  - (np.abs(s) ** 2 / n)[:, None] * c_hat)


def backward(theta, cache, g: np.ndarray, Q: int, hidden: int = HIDDEN) -> np.ndarray:
    """Gradient of sum over voxels of L w.r.t. theta, given g = dL/dc_hat
    (complex, as from loss_grad) per voxel."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, Q, hidden)
    z, a1, h1, a2, h2 = cache
    dy = np.empty((len(g), 2 * Q))
    dy[:, 0::2] = g.real
    dy[:, 1::2] = g.imag
    dW3 = dy.T @ h2
    db3 = dy.sum(0)
    dh2 = (dy @ W3) * (a2 > 0)
    dW2 = dh2.T @ h1
    db2 = dh2.sum(0)
    dh1 = (dh2 @ W2) * (a1 > 0)
    dW1 = dh1.T @ z
    db1 = dh1.sum(0)
    return np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3.ravel(), db3])


def batch_loss_and_grad(theta, G, nb, c, bound, Q: int, hidden: int = HIDDEN):
    """Mean loss over the batch and its gradient."""
    z = features(G, nb, bound)
    c_hat, cache = forward(theta, z, nb, Q, hidden)
    L = loss(c_hat, c)
    grad = backward(theta, cache, loss_grad(c_hat, c), Q, hidden)
    return float(L.mean()), grad / len(L)


def adam_step(theta, m, v, grad, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015) with bias correction; step >= 1."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
