"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these retypes an oracle formula: each compares the oracle with an
independent route (an explicit matrix, a brute-force sum, an SVD, a closed
form, a known lattice count or an invariant), chosen so that a dropped term,
a wrong sign, a transposed operand or an off-by-one index fails.
"""
import os

import numpy as np
import pytest

from oracle import calib, eig, gx, lagkernel, llr, maps, metrics, nullspace, support
from synth import generator, workloads

HERE = os.path.dirname(os.path.abspath(__file__))


def _tiny_acs(seed=3, Q=3, A=(10, 10), snr=40.0, grid=(24, 24)):
    sc = generator.make_scan(seed, grid, Q, A, 3, snr)
    return sc


# ---------------------------------------------------------------- support


def test_support_counts_match_lattice_table():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "lattice_counts.txt"))
            if l.strip() and not l.startswith("#")]
    for D, r, cnt in rows:
        lam = support.kernel_support(int(D), float(r))
        assert len(lam) == int(cnt), (D, r)


def test_support_order_and_shape():
    lam = support.kernel_support(2, 2.0)
    # lexicographic, last coordinate fastest
    keys = [tuple(v) for v in lam]
    assert keys == sorted(keys)
    assert (0, 0) in keys and (0, 2) in keys and (2, 0) in keys
    assert (1, 2) not in keys  # 1 + 4 > 4
    rect = support.kernel_support(2, 2.0, "rectangle")
    assert len(rect) == 25


def test_difference_set_brute_force():
    lam = support.kernel_support(2, 3.0)
    lags = support.difference_set(lam)
    brute = set()
    for a in range(len(lam)):
        for b in range(len(lam)):
            brute.add(tuple(lam[a] - lam[b]))
    assert set(map(tuple, lags)) == brute
    # symmetric under negation and contained in the ball of radius 2 tau
    s = set(map(tuple, lags))
    assert all(tuple(-np.array(v)) in s for v in s)
    assert np.all((lags ** 2).sum(1) <= 36)


# ---------------------------------------------------------------- Gram (Sec. IV-A)


@pytest.mark.parametrize("D,A,radius", [(2, (9, 11), 2.0), (3, (6, 5, 7), 1.5)])
def test_lag_gram_equals_explicit_cfull(D, A, radius):
    rng = np.random.default_rng(11)
    Q = 3
    acs = rng.standard_normal((Q,) + A) + 1j * rng.standard_normal((Q,) + A)
    lam = support.kernel_support(D, radius)
    lags = support.difference_set(lam)
    R = calib.correlation_lags(acs, lags)
    gram = calib.gram_from_lags(R, lam, lags)
    C = calib.calibration_matrix(acs, lam, "full")
    ref = C.conj().T @ C
    assert np.max(np.abs(gram - ref)) <= 1e-13 * np.max(np.abs(ref))
    # masking matters: the valid-row Gram is different (reported, not pinned)
    Cv = calib.calibration_matrix(acs, lam, "valid")
    assert Cv.shape[0] == int(np.prod([a - 2 * int(radius) for a in A]))
    assert np.max(np.abs(Cv.conj().T @ Cv - ref)) > 1e-3 * np.max(np.abs(ref))


@pytest.mark.parametrize("D,A,radius,shape", [(2, (12, 11), 2.0, "ellipsoid"),
                                               (2, (10, 10), 2.0, "rectangle"),
                                               (3, (8, 9, 8), 1.5, "ellipsoid")])
def test_valid_rows_gram(D, A, radius, shape):
    """C_valid (Sec. IV-A's masked form): prod(A - 2 tau) rows, each row's
    neighbourhood inside the ACS.  A row n outside C_valid has some n - n_i
    outside the ACS along a coordinate, so every other entry n - n_j lies
    within 2 tau of the border along it: when every sample within 2 tau of
    the border is zero, those rows are all zero and C_valid^H C_valid equals
    the correlation Gram (C_full^H C_full) exactly; otherwise it differs."""
    rng = np.random.default_rng(31)
    Q = 3
    lam = support.kernel_support(D, radius, shape)
    lags = support.difference_set(lam)
    tau = int(np.floor(radius))
    acs = rng.standard_normal((Q,) + A) + 1j * rng.standard_normal((Q,) + A)
    Cv = calib.calibration_matrix(acs, lam, rows="valid")
    assert Cv.shape == (int(np.prod([a - 2 * tau for a in A])), Q * len(lam))
    full = calib.gram_from_lags(calib.correlation_lags(acs, lags), lam, lags)
    assert np.abs(Cv.conj().T @ Cv - full).max() > 1e-3 * np.abs(full).max()
    inner = acs.copy()
    for d in range(D):
        sl = [slice(None)] * (D + 1)
        sl[d + 1] = slice(0, 2 * tau)
        inner[tuple(sl)] = 0
        sl[d + 1] = slice(A[d] - 2 * tau, A[d])
        inner[tuple(sl)] = 0
    assert np.abs(inner).max() > 0
    Cv = calib.calibration_matrix(inner, lam, rows="valid")
    full = calib.gram_from_lags(calib.correlation_lags(inner, lags), lam, lags)
    assert np.abs(Cv.conj().T @ Cv - full).max() <= 1e-13 * np.abs(full).max()


def test_gram_closed_forms():
    sc = _tiny_acs()
    acs = sc.acs
    Q = acs.shape[0]
    lam = support.kernel_support(2, 2.0)
    lags = support.difference_set(lam)
    R = calib.correlation_lags(acs, lags)
    gram = calib.gram_from_lags(R, lam, lags)
    assert np.allclose(gram, gram.conj().T, atol=0, rtol=0) or \
        np.max(np.abs(gram - gram.conj().T)) < 1e-12 * np.abs(gram).max()
    energy = np.sum(np.abs(acs) ** 2)
    assert np.isclose(np.trace(gram).real, len(lam) * energy, rtol=1e-13)
    zero = [i for i, v in enumerate(lags) if not v.any()][0]
    flat = acs.reshape(Q, -1)
    assert np.allclose(R[:, :, zero], flat.conj() @ flat.T, rtol=1e-13, atol=0)
    # Hermitian lag symmetry R_qp[-d] = conj(R_pq[d])
    idx = support.index_of(lags)
    for l, d in enumerate(lags):
        m = idx[tuple(-d)]
        assert np.allclose(R[:, :, m].T, R[:, :, l].conj(), rtol=1e-13, atol=1e-13)


def test_correlation_matches_fft_route():
    """Sec. IV-A: zero-padded FFTs give the same lags (exact in exact
    arithmetic) once the pad is at least A + 2 tau."""
    rng = np.random.default_rng(5)
    Q, A, tau = 2, (8, 8), 2
    acs = rng.standard_normal((Q,) + A) + 1j * rng.standard_normal((Q,) + A)
    lam = support.kernel_support(2, float(tau))
    lags = support.difference_set(lam)
    R = calib.correlation_lags(acs, lags)
    L = A[0] + 2 * tau
    S = np.fft.fft2(acs, s=(L, L))
    for p in range(Q):
        for q in range(Q):
            r = np.fft.ifft2(np.conj(S[p]) * S[q])
            for l, d in enumerate(lags):
                assert abs(r[d[0] % L, d[1] % L] - R[p, q, l]) < 1e-12


# ---------------------------------------------------------------- nullspace (Sec. III-A/B)


def test_nullspace_projector_matches_svd_of_c():
    sc = _tiny_acs(seed=21, Q=3, A=(12, 12))
    lam = support.kernel_support(2, 2.0)
    lags = support.difference_set(lam)
    gram = calib.gram_from_lags(calib.correlation_lags(sc.acs, lags), lam, lags)
    sp = nullspace.split_from_gram(gram)
    assert sp.gap >= 1e-3, "threshold-ambiguous instance; reseed"
    C = calib.calibration_matrix(sc.acs, lam, "full")
    sig, V, r_s = nullspace.split_from_svd(C)
    assert r_s == sp.r_signal
    assert np.allclose(np.sqrt(sp.eigvals), sig, rtol=1e-9, atol=1e-10 * sig[0])
    Pn = nullspace.projector(sp.null)
    Pn_svd = nullspace.projector(V[:, r_s:])
    assert np.max(np.abs(Pn - Pn_svd)) < 1e-10


def test_nullspace_orthonormal_and_residual():
    sc = _tiny_acs(seed=22, Q=3, A=(12, 12))
    lam = support.kernel_support(2, 2.0)
    lags = support.difference_set(lam)
    gram = calib.gram_from_lags(calib.correlation_lags(sc.acs, lags), lam, lags)
    sp = nullspace.split_from_gram(gram)
    V = sp.vectors
    assert np.max(np.abs(V.conj().T @ V - np.eye(len(V)))) < 1e-12
    res = gram @ V - V * sp.eigvals[None, :]
    assert np.max(np.linalg.norm(res, axis=0)) < 1e-11 * sp.eigvals[0]
    assert np.all(np.diff(sp.eigvals) <= 0)
    thr = 0.05 ** 2 * sp.eigvals[0]
    assert np.all(sp.eigvals[: sp.r_signal] >= thr)
    assert np.all(sp.eigvals[sp.r_signal:] < thr)


# ---------------------------------------------------------------- lag kernel (Eqs. 25-26)


def _small_problem(seed=31, Q=3, A=(12, 12), tau=2.0):
    sc = _tiny_acs(seed=seed, Q=Q, A=A)
    lam = support.kernel_support(2, tau)
    lags = support.difference_set(lam)
    gram = calib.gram_from_lags(calib.correlation_lags(sc.acs, lags), lam, lags)
    return sc, lam, lags, nullspace.split_from_gram(gram)


def test_lag_kernel_identities():
    sc, lam, lags, sp = _small_problem()
    Q = sc.Q
    Kn = lagkernel.lag_kernel_from_filters(sp.null, lam, lags, Q)
    Ks = lagkernel.lag_kernel_from_filters(sp.signal, lam, lags, Q)
    idx = support.index_of(lags)
    zero = idx[(0, 0)]
    # Hermitian in (p, q, m): K_qp[-m] = conj(K_pq[m])
    for l, m in enumerate(lags):
        assert np.allclose(Kn[:, :, idx[tuple(-m)]].T, Kn[:, :, l].conj(), atol=1e-12)
    # trace of W equals the nullspace dimension R
    assert np.isclose(np.trace(Kn[:, :, zero]).real, sp.r_null, atol=1e-10)
    # complement (Eq. 20 route): K(null) + K(signal) = |Lambda| delta_pq delta[m]
    tot = Kn + Ks
    expect = np.zeros_like(tot)
    expect[:, :, zero] = len(lam) * np.eye(Q)
    assert np.max(np.abs(tot - expect)) < 1e-11


def test_lag_kernel_single_filter_brute_force():
    """For one filter, K_pq[m] is the cross-correlation
    sum_s conj(h[n_s + m, p]) h[n_s, q]; checked by direct loops."""
    rng = np.random.default_rng(2)
    Q = 2
    lam = support.kernel_support(2, 1.0)
    lags = support.difference_set(lam)
    h = rng.standard_normal((Q * len(lam), 1)) + 1j * rng.standard_normal((Q * len(lam), 1))
    K = lagkernel.lag_kernel_from_filters(h, lam, lags, Q)
    pos = support.index_of(lam)
    for l, m in enumerate(lags):
        for p in range(Q):
            for q in range(Q):
                acc = 0
                for s, ns in enumerate(lam):
                    t = pos.get(tuple(ns + m))
                    if t is not None:
                        acc += np.conj(h[p * len(lam) + t, 0]) * h[q * len(lam) + s, 0]
                assert abs(acc - K[p, q, l]) < 1e-13


# ---------------------------------------------------------------- G(x) (Eqs. 15-26)


def test_gx_three_forms_agree_off_grid():
    sc, lam, lags, sp = _small_problem()
    Q = sc.Q
    rng = np.random.default_rng(9)
    x = rng.uniform(-0.5, 0.5, size=(7, 2))
    Kn = lagkernel.lag_kernel_from_filters(sp.null, lam, lags, Q)
    g_k = gx.gx_from_lag_kernel(Kn, lags, x)
    g_24 = gx.gx_eq24(sp.null, lam, x, Q)
    g_h = gx.gx_from_filters(sp.null, lam, x, Q)
    scale = len(lam)
    assert np.max(np.abs(g_k - g_h)) < 1e-12 * scale
    assert np.max(np.abs(g_24 - g_h)) < 1e-12 * scale


def test_gx_spectrum_bounds_and_dc_identity():
    sc, lam, lags, sp = _small_problem()
    Q = sc.Q
    Kn = lagkernel.lag_kernel_from_filters(sp.null, lam, lags, Q)
    grid = (9, 9)                      # >= 4 tau + 1 with tau = 2
    x = gx.grid_points(grid)
    G = gx.gx_from_lag_kernel(Kn, lags, x)
    assert np.max(np.abs(G - np.conj(np.transpose(G, (0, 2, 1))))) < 1e-12
    w = np.linalg.eigvalsh(G)
    assert w.min() > -1e-10 and w.max() < len(lam) + 1e-10
    mean_tr = np.mean(np.real(np.einsum("xqq->x", G)))
    assert np.isclose(mean_tr, sp.r_null, rtol=1e-12)
    # complement: G(null) + G(signal) = |Lambda| I at every x (Eq. 20)
    Ks = lagkernel.lag_kernel_from_filters(sp.signal, lam, lags, Q)
    Gs = gx.gx_from_lag_kernel(Ks, lags, x)
    assert np.max(np.abs(G + Gs - len(lam) * np.eye(Q)[None])) < 1e-11


# ---------------------------------------------------------------- end-to-end exact case (Eqs. 9-11)


def test_exact_annihilator_recovers_maps():
    """Noiseless data, maps that are trigonometric polynomials with Fourier
    support inside Lambda and an image with no zeros: the cross-relation
    filters of Eq. (11) annihilate the data exactly, so c(x) is an exact null
    vector of G(x) built from the valid-row C (no implicit zeros)."""
    rng = np.random.default_rng(4)
    Q, D, N, A, tau = 4, 2, 32, 20, 2.0
    lam = support.kernel_support(D, tau)
    ax = (np.arange(N) - N // 2) / N
    X, Y = np.meshgrid(ax, ax, indexing="ij")
    rho = (2.0 + 0.5 * np.cos(2 * np.pi * X) + 0.3j * np.sin(2 * np.pi * (X + 2 * Y)))
    B = [(0, 0), (0, 1), (1, 0), (-1, 0), (0, -1)]
    cmaps = np.zeros((Q, N, N), dtype=np.complex128)
    for q in range(Q):
        for b in B:
            coef = rng.standard_normal() + 1j * rng.standard_normal()
            cmaps[q] += coef * np.exp(2j * np.pi * (b[0] * X + b[1] * Y))
    coil = cmaps * rho[None]
    ksp = generator.centred_fft(coil, (1, 2))
    acs = generator.centre_block(ksp, (A, A))
    C = calib.calibration_matrix(acs, lam, "valid")
    gram = C.conj().T @ C
    sp = nullspace.split_from_gram(gram, thresh=1e-7)
    lags = support.difference_set(lam)
    Kn = lagkernel.lag_kernel_from_filters(sp.null, lam, lags, Q)
    pts = gx.grid_points((N, N))
    G = gx.gx_from_lag_kernel(Kn, lags, pts)
    ctrue = cmaps.reshape(Q, -1).T
    lmin, cmin, l2 = eig.smallest_exact(G)
    good = np.linalg.norm(ctrue, axis=1) > 1e-3 * np.linalg.norm(ctrue, axis=1).max()
    resid = np.linalg.norm(np.einsum("xpq,xq->xp", G, ctrue), axis=1) / np.linalg.norm(ctrue, axis=1)
    assert np.max(resid[good]) < 1e-8 * len(lam)
    err = metrics.map_error(ctrue.T, cmin.T, axis=0)
    assert np.max(err[good]) < 1e-6
    assert np.min(l2[good]) > 1e-4 * len(lam)


# ---------------------------------------------------------------- per-voxel eigenvectors (Sec. IV-E)


def _random_psd_field(rng, Nv, Q, bound, gap=0.3):
    U = np.linalg.qr(rng.standard_normal((Nv, Q, Q)) + 1j * rng.standard_normal((Nv, Q, Q)))[0]
    w = np.sort(rng.uniform(gap, 1.0, size=(Nv, Q)), axis=1) * bound
    w[:, 0] = rng.uniform(0, 0.02, size=Nv) * bound
    return np.einsum("xpk,xk,xqk->xpq", U, w, U.conj()), U, w


def test_exact_eig_q2_closed_form():
    a, c, b = 3.0, 1.0, 1.0 + 2.0j
    G = np.array([[[a, b], [np.conj(b), c]]])
    lmin, v, _ = eig.smallest_exact(G)
    closed = 0.5 * (a + c) - np.sqrt(0.25 * (a - c) ** 2 + abs(b) ** 2)
    assert np.isclose(lmin[0], closed, rtol=1e-14)
    assert np.allclose(G[0] @ v[0], closed * v[0], atol=1e-13)


def test_power_iteration_bound_and_convergence():
    rng = np.random.default_rng(1)
    Q, bound = 6, 10.0
    G, U, w = _random_psd_field(rng, 50, Q, bound)
    lmin, cmin, _ = eig.smallest_exact(G)
    for k in (3, 10, 30):
        c, lam, r, it = eig.power_iteration(G, bound, k)
        assert np.allclose(np.linalg.norm(c, axis=1), 1.0, atol=1e-14)
        assert np.all(it == k)
        # textbook bound: sin of the angle <= tan(angle0) (mu2/mu1)^k for Gs
        mu = np.sort(bound - w, axis=1)[:, ::-1]
        q0 = eig.initial_index(G)
        cos0 = np.abs(cmin[np.arange(len(q0)), q0])
        tan0 = np.sqrt(np.maximum(1 - cos0 ** 2, 0)) / cos0
        bnd = tan0 * (mu[:, 1] / mu[:, 0]) ** k
        ip = np.sum(np.conj(cmin) * c, axis=1)
        sin = np.linalg.norm(c - ip[:, None] * cmin, axis=1)
        assert np.all(sin <= bnd * (1 + 1e-9) + 1e-12)
    c, lam, r, it = eig.power_iteration(G, bound, tol=1e-12, max_iter=400)
    assert np.all(r <= 1e-12 * bound)
    assert np.allclose(lam, lmin, atol=1e-10 * bound)


def test_smallest_set_recovers_constructed_spectrum():
    """G = U diag(w) U^H with a known unitary U and known eigenvalues (two
    near zero, as under aliasing): the M smallest pairs are the constructed
    ones, in ascending order, up to a phase per vector."""
    rng = np.random.default_rng(22)
    Nv, Q, bound = 30, 6, 10.0
    U = np.linalg.qr(rng.standard_normal((Nv, Q, Q)) + 1j * rng.standard_normal((Nv, Q, Q)))[0]
    w = np.sort(rng.uniform(2.0, 9.0, size=(Nv, Q)), axis=1)
    w[:, 0] = rng.uniform(0, 1e-3, Nv)
    w[:, 1] = w[:, 0] + rng.uniform(0.05, 0.2, Nv)
    G = np.einsum("xpk,xk,xqk->xpq", U, w, U.conj())
    lam, c = eig.smallest_set(G, 3)
    assert np.allclose(lam, w[:, :3], atol=1e-12 * bound)
    for m in range(3):
        ov = np.abs(np.einsum("xq,xq->x", U[:, :, m].conj(), c[:, :, m]))
        assert np.allclose(ov, 1.0, atol=1e-10)
    l1, c1, _ = eig.smallest_exact(G)
    assert np.allclose(l1, lam[:, 0], atol=1e-12 * bound)


def test_partial_svd_pins():
    """Partial SVDs: a patch of exact rank r is reproduced to rounding; for
    any patch the truncation error in the Frobenius norm is the root sum of
    squares of the dropped singular values (Eckart-Young); the singular
    values of a matrix built from known orthonormal factors are returned."""
    rng = np.random.default_rng(23)
    B, Q, m, r = 20, 6, 16, 2
    A = rng.standard_normal((B, m, r)) + 1j * rng.standard_normal((B, m, r))
    C = rng.standard_normal((B, r, Q)) + 1j * rng.standard_normal((B, r, Q))
    X = np.transpose(A @ C, (0, 2, 1))
    s, V, Xr = llr.partial_svd(X, r)
    assert np.abs(Xr - X).max() <= 1e-12 * np.abs(X).max()
    X = rng.standard_normal((B, Q, m)) + 1j * rng.standard_normal((B, Q, m))
    s_all = np.linalg.svd(np.transpose(X, (0, 2, 1)), compute_uv=False)
    s, V, Xr = llr.partial_svd(X, r)
    err = np.linalg.norm((X - Xr).reshape(B, -1), axis=1)
    assert np.allclose(err, np.sqrt(np.sum(s_all[:, r:] ** 2, axis=1)), rtol=1e-10)
    Uo = np.linalg.qr(rng.standard_normal((B, m, Q)) + 1j * rng.standard_normal((B, m, Q)))[0]
    Vo = np.linalg.qr(rng.standard_normal((B, Q, Q)) + 1j * rng.standard_normal((B, Q, Q)))[0]
    sig = np.sort(rng.uniform(0.1, 2.0, (B, Q)), axis=1)[:, ::-1]
    M = np.einsum("bik,bk,bqk->biq", Uo, sig, Vo.conj())
    s, V, _ = llr.partial_svd(np.transpose(M, (0, 2, 1)), 3)
    assert np.allclose(s, sig[:, :3], rtol=1e-12)
    ov = np.abs(np.einsum("bqk,bqk->bk", Vo[:, :, :3].conj(), V))
    assert np.allclose(ov, 1.0, atol=1e-9)


def test_rayleigh_check():
    """The Rayleigh check (Sec. IV-E): on exact eigenvectors (numpy eigh)
    it returns their eigenvalue with a residual at rounding level; for a
    perturbed vector c = u1 + e u2 of a diagonal G the closed forms
    lambda = (l1 + e^2 l2)/(1 + e^2) and residual e |l2 - l1| / (1 + e^2)
    hold; it is invariant to the scale and phase of c."""
    rng = np.random.default_rng(21)
    Q, bound = 7, 20.0
    G, U, w = _random_psd_field(rng, 40, Q, bound)
    lmin, cmin, _ = eig.smallest_exact(G)
    lam, r = eig.rayleigh(G, cmin)
    assert np.allclose(lam, lmin, atol=1e-13 * bound)
    assert np.all(r <= 1e-13 * bound)
    lam2, r2 = eig.rayleigh(G, cmin * (3.0 * np.exp(1j * rng.uniform(0, 6, (40, 1)))))
    assert np.allclose(lam2, lam, atol=1e-13 * bound) and np.allclose(r2, r, atol=1e-13 * bound)
    l1, l2, e = 2.0, 5.0, 0.3
    D = np.diag([l1, l2, 9.0]).astype(complex)[None]
    c = np.array([[1.0, e, 0.0]], dtype=complex)
    lam3, r3 = eig.rayleigh(D, c)
    assert np.isclose(lam3[0], (l1 + e * e * l2) / (1 + e * e), rtol=1e-14)
    assert np.isclose(r3[0], e * abs(l2 - l1) / (1 + e * e), rtol=1e-13)


# ---------------------------------------------------------------- phase, interpolation, normalisation


def test_apodized_lowres_matches_inverse_fft_without_apodization():
    """With the grid equal to the ACS size, the Gaussian-weighted sum with the
    weights divided out is the centred inverse DFT (numpy) times sqrt(N)."""
    rng = np.random.default_rng(8)
    Q, A = 2, (8, 6)
    acs = rng.standard_normal((Q,) + A) + 1j * rng.standard_normal((Q,) + A)
    gw = [np.exp(-((np.arange(a) - a // 2) ** 2) / (2 * (a / 4.0) ** 2)) for a in A]
    g = np.outer(gw[0], gw[1])
    out = maps.apodized_lowres(acs / g[None], A)
    ref = generator.centred_ifft(acs, (1, 2)) * np.sqrt(np.prod(A))
    assert np.allclose(out, ref, atol=1e-12)


def test_phase_reference_makes_combination_real_positive():
    rng = np.random.default_rng(12)
    Q, grid = 4, (6, 5)
    c = rng.standard_normal((Q,) + grid) + 1j * rng.standard_normal((Q,) + grid)
    c /= np.linalg.norm(c, axis=0, keepdims=True)
    rho = rng.standard_normal((Q,) + grid) + 1j * rng.standard_normal((Q,) + grid)
    c2, alpha = maps.phase_reference(c, rho)
    m = np.sum(np.conj(c2) * rho, axis=0)
    assert np.max(np.abs(m.imag)) < 1e-14 * np.abs(m).max()
    assert np.all(m.real >= 0)
    assert np.allclose(np.abs(alpha), 1.0)
    assert np.allclose(np.abs(c2), np.abs(c))


def test_interpolation_reproduces_samples_and_trig_polynomials():
    rng = np.random.default_rng(13)
    Q = 2
    lr, out = (8, 6), (24, 18)
    c = rng.standard_normal((Q,) + lr) + 1j * rng.standard_normal((Q,) + lr)
    up = maps.interpolate(c, out)
    # coarse points sit at every 3rd output point (centred grids)
    sub = up[:, (np.arange(lr[0]) - lr[0] // 2) * 3 + out[0] // 2][:, :, (np.arange(lr[1]) - lr[1] // 2) * 3 + out[1] // 2]
    assert np.allclose(sub, c, atol=1e-12)
    # band-limited trig polynomial reproduced at any output size
    ks = [(1, -2), (-3, 2), (0, 0)]
    coef = rng.standard_normal(len(ks)) + 1j * rng.standard_normal(len(ks))

    def f(grid):
        ax = [(np.arange(n) - n // 2) / n for n in grid]
        X, Y = np.meshgrid(*ax, indexing="ij")
        return sum(a * np.exp(2j * np.pi * (k[0] * X + k[1] * Y)) for a, k in zip(coef, ks))

    for o in [(17, 13), (32, 32)]:
        got = maps.interpolate(f(lr)[None], o)[0]
        assert np.allclose(got, f(o), atol=1e-12)
    # linear
    d = rng.standard_normal((Q,) + lr)
    assert np.allclose(maps.interpolate(c + 2 * d, out), up + 2 * maps.interpolate(d, out), atol=1e-12)


def test_interpolation_nyquist_split_is_real_preserving():
    """An even-length real signal must stay real after upsampling; this fails
    if the Nyquist coefficient is kept on one side only."""
    rng = np.random.default_rng(14)
    c = rng.standard_normal((1, 8))
    T = maps.sinc_matrix(8, 20)
    assert np.max(np.abs((T @ c[0]).imag)) < 1e-13


def test_normalize_rss():
    rng = np.random.default_rng(15)
    c = rng.standard_normal((3, 4, 4)) + 1j * rng.standard_normal((3, 4, 4))
    c[:, 0, 0] = 0
    n = maps.normalize_rss(c)
    rss = np.sqrt(np.sum(np.abs(n) ** 2, axis=0))
    assert np.all(n[:, 0, 0] == 0)
    rss[0, 0] = 1
    assert np.allclose(rss, 1.0)


# ---------------------------------------------------------------- metrics and generator


def test_projection_residual_and_map_error():
    sc = generator.make_scan(5, (32, 32), 4, (12, 12), 3, 200.0)
    coil = sc.maps * sc.image[None]
    assert metrics.projection_residual(coil, sc.maps) < 1e-12
    phase = np.exp(1j * np.random.default_rng(0).uniform(0, 6, size=(32, 32)))
    assert metrics.projection_residual(coil, sc.maps * phase[None] * 3.0) < 1e-12
    assert np.max(metrics.map_error(sc.maps, sc.maps * phase[None])) < 1e-7
    flat = np.ones_like(sc.maps)
    r = metrics.projection_residual(coil, flat)
    assert 0.05 < r < 1.0


def test_generator_properties():
    w = workloads.SMALL_2D
    a = w.scan()
    b = w.scan()
    assert np.array_equal(a.acs, b.acs)
    rss = np.sqrt(np.sum(np.abs(a.maps) ** 2, axis=0))
    assert np.allclose(rss, 1.0)
    coil = a.maps * a.image[None]
    noise = a.kspace - generator.centred_fft(coil, (1, 2))
    snr = 10 * np.log10(np.mean(np.abs(coil) ** 2) / np.mean(np.abs(noise) ** 2))
    assert abs(snr - w.snr_db) < 0.1
    ax = (np.arange(64) - 32) / 64
    X, Y = np.meshgrid(ax, ax, indexing="ij")
    assert np.all(a.image[np.maximum(abs(X), abs(Y)) > 0.45] == 0)
    assert a.acs.shape == (8, 24, 24)
    # ACS index a <-> k = a - floor(A/2): the DC sample is at the centre
    assert np.allclose(a.acs[:, 12, 12], a.kspace[:, 32, 32])


def test_map_error_has_no_cancellation_floor():
    """Unit b = (a cos t + w sin t) e^{i psi} with w orthogonal to a has the
    closed-form distance 2 sin(t/2); it must be resolved down to 1e-9, far
    below the sqrt(eps) floor of the 2 - 2|a^H b| form."""
    rng = np.random.default_rng(3)
    a = rng.standard_normal((10, 5)) + 1j * rng.standard_normal((10, 5))
    a = metrics.unit(a)
    w = rng.standard_normal((10, 5)) + 1j * rng.standard_normal((10, 5))
    w = metrics.unit(w - a * np.sum(np.conj(a) * w, axis=0, keepdims=True))
    t = np.array([1e-9, 3e-8, 1e-6, 1e-3, 0.5])
    b = (a * np.cos(t) + w * np.sin(t)) * np.exp(1j * np.array([0.3, 1.3, 2.0, -1.0, 3.0]))
    e = metrics.map_error(a, b)
    assert np.allclose(e, 2 * np.sin(t / 2), rtol=1e-6, atol=0)


# ---------------------------------------------------------------- start vector, coil reference


def test_initial_index_picks_smallest_diagonal_lowest_on_ties():
    """q* = argmin diag G(x), lowest index on ties: a constructed field where
    argmax, the last minimum, or the off-diagonal would pick another index."""
    Q = 5
    diag = np.array([
        [3.0, 1.0, 2.0, 5.0, 4.0],    # unique minimum at 1
        [2.0, 0.5, 0.5, 9.0, 0.5],    # three-way tie at 1, 2, 4 -> 1
        [7.0, 7.0, 7.0, 7.0, 7.0],    # all equal -> 0
        [4.0, 4.0, 4.0, 4.0, 0.25],   # minimum last -> 4
    ])
    G = np.zeros((len(diag), Q, Q), dtype=np.complex128)
    for x, d in enumerate(diag):
        G[x] = np.diag(d)
        # large off-diagonal entries must not influence the choice
        G[x, 0, 3] = 50.0 + 20.0j
        G[x, 3, 0] = 50.0 - 20.0j
    q = eig.initial_index(G)
    assert list(q) == [1, 1, 0, 4]
    # the start vector the iteration uses is e_{q*}: zero steps return it
    c, _, _, it = eig.power_iteration(G, 100.0, n_iter=0)
    assert np.all(it == 0)
    ref = np.zeros((len(diag), Q))
    ref[np.arange(len(diag)), [1, 1, 0, 4]] = 1.0
    assert np.array_equal(c, ref)


def test_coil_reference_rule():
    """Sec. V rule: after referencing, the reference channel is real and
    non-negative, magnitudes are unchanged, and the result does not depend on
    a per-voxel phase of the input; a voxel whose reference entry is zero is
    left unchanged."""
    rng = np.random.default_rng(21)
    Q, grid = 4, (5, 6)
    c = rng.standard_normal((Q,) + grid) + 1j * rng.standard_normal((Q,) + grid)
    c[0, 1, 2] = 0.0
    out = maps.coil_reference(c)
    nz = np.abs(c[0]) > 0
    assert np.all(np.abs(out[0][nz].imag) <= 1e-15 * np.abs(out[0][nz]))
    assert np.all(out[0][nz].real > 0)
    assert np.allclose(np.abs(out), np.abs(c), rtol=1e-15, atol=0)
    assert np.array_equal(out[:, 1, 2], c[:, 1, 2])
    phase = np.exp(1j * rng.uniform(0, 2 * np.pi, size=grid))
    again = maps.coil_reference(c * phase[None])
    assert np.allclose(again[:, nz], out[:, nz], atol=1e-14)
    # another reference channel
    out2 = maps.coil_reference(c, q_ref=2)
    assert np.all(np.abs(out2[2].imag) <= 1e-15 * np.abs(out2[2]))
    assert np.all(out2[2].real > 0)
    # closed form for Q = 2: (r e^{ia}, s e^{ib}) -> (r, s e^{i(b - a)})
    two = np.array([[2.0 * np.exp(0.7j)], [3.0 * np.exp(-1.1j)]])
    assert np.allclose(maps.coil_reference(two), [[2.0], [3.0 * np.exp(-1.8j)]], atol=1e-15)


# ---------------------------------------------------------------- end to end (P-R1)


def _recovery(sc, radius, grid_lr):
    from scipy import ndimage
    from oracle import pipeline
    acs = generator.as_device_input(sc.acs)
    res = pipeline.estimate(acs, radius, grid_lr, sc.grid)
    inner = ndimage.binary_erosion(np.abs(sc.image) > 0, iterations=2)
    e = metrics.map_error(sc.maps, res.maps)[inner]
    axes = tuple(range(1, sc.image.ndim + 1))
    coil_noisy = generator.centred_ifft(sc.kspace, axes)
    return res, e, coil_noisy


@pytest.mark.parametrize("seed", [1000, 1002])
def test_pipeline_recovers_generator_maps_2d(seed):
    """The whole oracle pipeline (C_full Gram, eigen split, lag kernel, G(x),
    power iteration, phase reference, interpolation, RSS) on a seeded scan
    of the 64^2, 8-coil, 24^2-ACS family recovers the generator's maps up to
    the per-voxel scale (Sec. II) on the object eroded by two voxels.  The
    maps are smooth but not band-limited, so recovery is approximate: on the
    full-resolution estimation grid the median distance is below 1e-2; on the
    workload's 32^2 grid, interpolation adds a few 1e-2 (Sec. IV-D).  A
    wrong sign, lag or transposed block gives distances of order one."""
    w = workloads.SMALL_2D
    sc = w.scan(seed)
    res, e, coil = _recovery(sc, w.radius, sc.grid)
    assert np.median(e) <= 1e-2
    assert np.percentile(e, 90) <= 2.5e-2
    # the projection residual sits near the noise floor (the residual of the
    # true maps is the noise's share of the data)
    r_est = metrics.projection_residual(coil, res.maps)
    r_true = metrics.projection_residual(coil, sc.maps)
    assert r_true <= r_est <= 2.0 * r_true
    # Table I pattern: ESPIRiT-form maps (top eigenvector of the operator
    # built from the SIGNAL filters) give the same maps and the same residual
    x = gx.grid_points(sc.grid)
    Bs = gx.gx_from_filters(res.split.signal, res.lam, x, sc.Q) / len(res.lam)
    _, V = np.linalg.eigh(Bs)
    c_esp = V[:, :, -1].T.reshape(res.c_lr.shape)
    c_esp, _ = maps.phase_reference(c_esp, res.rho_lr)
    m_esp = maps.normalize_rss(maps.interpolate(c_esp, sc.grid))
    r_esp = metrics.projection_residual(coil, m_esp)
    _, c_ns, _ = eig.smallest_exact(res.G)
    c_ns, _ = maps.phase_reference(c_ns.T.reshape(res.c_lr.shape), res.rho_lr)
    r_ns = metrics.projection_residual(coil, maps.normalize_rss(maps.interpolate(c_ns, sc.grid)))
    assert abs(r_esp - r_ns) <= 1e-12 * r_ns
    # ten power-iteration steps (Sec. IV-E) change the residual only slightly
    assert abs(r_est - r_ns) <= 1e-4 * r_ns
    # the workload's own low-res grid
    _, e_lr, _ = _recovery(sc, w.radius, w.grid_lr)
    assert np.median(e_lr) <= 3e-2


def test_pipeline_recovers_generator_maps_3d():
    sc = generator.make_scan(7, (24, 24, 24), 4, (12, 12, 12), 5, 40.0)
    res, e, coil = _recovery(sc, 2.0, sc.grid)
    assert np.median(e) <= 2e-2
    assert np.percentile(e, 90) <= 3e-2
    r_est = metrics.projection_residual(coil, res.maps)
    r_true = metrics.projection_residual(coil, sc.maps)
    assert r_true <= r_est <= 4.0 * r_true


# ---------------------------------------------------------------- ESPIRiT operator, support mask


def test_espirit_operator_equals_signal_filter_form():
    """Eq. 20: I - G/|Lambda| built from the NULL filters equals the operator
    built from the SIGNAL filters, (1/|Lambda|) H_s^H H_s; its top eigenvector
    is G's bottom one."""
    sc = _tiny_acs(seed=4, Q=3)
    lam = support.kernel_support(2, 2.0)
    lags = support.difference_set(lam)
    gram = calib.gram_from_lags(calib.correlation_lags(sc.acs, lags), lam, lags)
    sp = nullspace.split_from_gram(gram)
    x = np.random.default_rng(5).uniform(-0.5, 0.5, size=(40, 2))
    G = gx.gx_from_filters(sp.null, lam, x, 3)
    B = gx.espirit_operator(G, len(lam))
    Bs = gx.gx_from_filters(sp.signal, lam, x, 3) / len(lam)
    assert np.max(np.abs(B - Bs)) <= 1e-12
    wB, VB = np.linalg.eigh(B)
    _, cmin, _ = eig.smallest_exact(G)
    assert np.max(metrics.map_error(VB[:, :, -1], cmin, axis=1)) <= 1e-7


def test_support_mask_separates_object_from_background():
    """Sec. III-D step 6 / Sec. III-B: lambda_min(G)/|Lambda| is near zero on
    the object and clearly positive off it; thresholding its interpolated map
    recovers the support away from the edges."""
    from scipy import ndimage
    from oracle import pipeline
    w = workloads.SMALL_2D
    sc = w.scan(1000)
    res = pipeline.estimate(generator.as_device_input(sc.acs), w.radius, w.grid_lr, sc.grid)
    obj = np.abs(sc.image) > 0
    inner = ndimage.binary_erosion(obj, iterations=2)
    outer = ~ndimage.binary_dilation(obj, iterations=2)
    m = maps.support_mask(res.lam_min.reshape(w.grid_lr), len(res.lam), sc.grid, 0.02)
    assert m.shape == sc.grid
    assert np.all(m[inner])
    assert np.mean(~m[outer]) >= 0.98
    # threshold monotone: a lower level keeps a subset
    m2 = maps.support_mask(res.lam_min.reshape(w.grid_lr), len(res.lam), sc.grid, 0.01)
    assert np.all(m[m2])
