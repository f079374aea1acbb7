"""Parity of every C-ABI stage with the FP64 oracle on the GPU.

Each stage is fed the same seeded input on both sides; oracle inputs come
from the generator or from the oracle itself, never from the HIP path.
Tolerances (errors vs FP64 are printed for every result):
  Gram            max|dG|/max|G| <= 1e-5 and ||dG||_F/||G||_F <= 1e-5
  eigenvalues     |d lambda_k| / lambda_1 <= 1e-5
  projector       max |P_gpu - P_oracle| <= 1e-7 (FP64 on the same matrix)
  G(x)            max|dG| / |Lambda| <= 1e-5
  lambda_min      |d lambda| / |Lambda| <= 1e-5
  maps            gauge-invariant e(x) <= 1e-4 where the map is defined
                  (coil-combined apodized image |m| >= 1e-3 max|m|, eroded by
                  one low-res voxel; elsewhere the phase reference divides
                  FP32 rounding by |m|, see the conditioning test).
"""
import numpy as np
import pytest

from oracle.metrics import map_error
from synth import generator, workloads

from .gpu_common import (lowres_mask, oeig, ogx, omaps, oracle_full, oracle_gram_split,
                         output_mask, packed_upper, lagkernel, sampled_points, scan_inputs)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

BLOCK = {"2d_64x64_q8_acs24_r3": 64, "2d_256x256_q32_acs32_r5": 96,
         "3d_96x160x160_q16_acs24_r4": 224}
WL2D = ["2d_64x64_q8_acs24_r3", "2d_256x256_q32_acs32_r5"]
WLALL = WL2D + ["3d_96x160x160_q16_acs24_r4"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2302_13431_amd  # noqa: F401


def estimator(name, **kw):
    import paper_2302_13431_amd as P
    w = workloads.ALL[name]
    kw.setdefault("block", BLOCK[name])
    return P.Estimator(w.Q, w.acs, w.radius, w.grid_lr, w.grid, **kw)


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def report(tag, **vals):
    print(f"[{tag}] " + " ".join(f"{k}={v:.3e}" if isinstance(v, float) else f"{k}={v}"
                                 for k, v in vals.items()), flush=True)


# ------------------------------------------------------------------ Gram


@pytest.mark.parametrize("name", WLALL)
def test_gram(name):
    w, acs = scan_inputs(name)
    _, _, gram, _, _ = oracle_gram_split(name)
    est = estimator(name)
    g = est.gram(cuda(acs)).cpu().numpy().astype(np.complex128)
    e_max = float(np.abs(g - gram).max() / np.abs(gram).max())
    e_fro = float(np.linalg.norm(g - gram) / np.linalg.norm(gram))
    report("gram " + name, err_max=e_max, err_fro=e_fro)
    assert np.array_equal(g, g.conj().T)
    assert e_max <= 1e-5 and e_fro <= 1e-5
    assert est.status() == 0


@pytest.mark.parametrize("acs_n", [40, 64])
def test_gram_fft_lengths(acs_n):
    """The correlation's inverse passes at F = 64 (column blocks, pairs split
    over workgroups) and F = 128 (the line-per-pair passes that take F above
    64): ACS 40 and 64 with radius 3 give F = next_pow2(A + 6) = 64 and 128.
    Random channels (the Gram is defined for any data), oracle Gram from the
    correlation lags."""
    import paper_2302_13431_amd as P
    from oracle import calib, support
    Q, radius = 8, 3.0
    rng = np.random.default_rng(1000 + acs_n)
    acs = (rng.standard_normal((Q, acs_n, acs_n))
           + 1j * rng.standard_normal((Q, acs_n, acs_n))).astype(np.complex64)
    lam = support.kernel_support(2, radius, "ellipsoid")
    lags = support.difference_set(lam)
    ref = calib.gram_from_lags(calib.correlation_lags(acs.astype(np.complex128), lags), lam,
                               lags)
    est = P.Estimator(Q, (acs_n, acs_n), radius, (32, 32), (64, 64), block=64)
    g = est.gram(cuda(acs)).cpu().numpy().astype(np.complex128)
    e_max = float(np.abs(g - ref).max() / np.abs(ref).max())
    e_fro = float(np.linalg.norm(g - ref) / np.linalg.norm(ref))
    report(f"gram fft lengths acs={acs_n}", err_max=e_max, err_fro=e_fro)
    assert np.array_equal(g, g.conj().T)
    assert e_max <= 1e-5 and e_fro <= 1e-5
    assert est.status() == 0


# ------------------------------------------------------------------ nullspace


NULL_CASES = [(w, BLOCK[w]) for w in WLALL] + [("2d_256x256_q32_acs32_r5", 128),
                                               ("2d_256x256_q32_acs32_r5", 160)]


@pytest.mark.parametrize("name,block", NULL_CASES)
def test_nullspace(name, block):
    """Blocks up to 96 are factored with the matrix in LDS, larger ones by
    the blocked (panel + multi-workgroup update) Cholesky; 128 and 160 also
    reach the register and global-memory tridiagonalisations."""
    _, _, _, g32, sp = oracle_gram_split(name)
    est = estimator(name, block=block)
    ev, basis, counts = est.nullspace(cuda(g32))
    ev, basis, counts = ev.cpu().numpy(), basis.cpu().numpy(), counts.cpu().numpy()
    rs = int(counts[0])
    report(f"nullspace {name} b={block}", r_gpu=rs, r_oracle=sp.r_signal,
           iters=int(counts[2]), gap=sp.gap)
    assert counts[3] == 1, "not converged"
    assert rs == sp.r_signal
    lam = sp.eigvals
    e_eig = float(np.abs(ev[:rs + 1] - lam[:rs + 1]).max() / lam[0])
    Vs = basis[:rs].T
    Po = sp.signal @ sp.signal.conj().T
    e_proj = float(np.abs(Vs @ Vs.conj().T - Po).max())
    e_orth = float(np.abs(basis.conj() @ basis.T - np.eye(len(basis))).max())
    report("nullspace " + name, err_eig=e_eig, err_proj=e_proj, err_orth=e_orth)
    assert e_eig <= 1e-5
    assert e_proj <= 1e-7
    assert e_orth <= 1e-10
    assert np.all(ev[rs:] < 0.05 ** 2 * ev[0]) and np.all(ev[:rs] >= 0.05 ** 2 * ev[0])


def test_nullspace_repeated_eigenvalues():
    """Gram with exactly repeated eigenvalues (a phase-permutation of a
    diagonal, exact in FP32): the Rayleigh-Ritz matrices then have clusters
    of equal eigenvalues, in the signal part and across the whole noise part
    of the block.  The signal projector is unique and must match; the basis
    must stay orthonormal.

    The iteration stops once every Ritz pair up to the first below threshold
    has residual <= 1e-10 theta_1; by the Davis-Kahan sin-theta theorem the
    signal projector then lies within ||R||_F / gap of the exact one, with
    ||R||_F <= sqrt(r + 1) 1e-10 theta_1 and gap = lambda_r - lambda_{r+1}.
    Both the residuals (in FP64 on the host) and that consequence are
    checked."""
    noise = 2.0 ** -10
    name = "2d_64x64_q8_acs24_r3"
    w = workloads.ALL[name]
    est = estimator(name)
    n = est.n
    rng = np.random.default_rng(11)
    vals = np.full(n, noise)
    vals[:20] = [100.0] * 10 + [40.0] * 5 + [1.0] * 5
    perm = rng.permutation(n)
    phase = np.array([1, -1, 1j, -1j])[rng.integers(0, 4, n)]
    Umat = np.zeros((n, n), complex)
    Umat[perm, np.arange(n)] = phase
    g = (Umat * vals) @ Umat.conj().T
    g32 = g.astype(np.complex64)
    assert np.array_equal(g32.astype(complex), g)
    ev, basis, counts = est.nullspace(cuda(g32))
    ev, basis, counts = ev.cpu().numpy(), basis.cpu().numpy(), counts.cpu().numpy()
    rs = int(counts[0])
    Vs = basis[:rs].T
    Po = Umat[:, :20] @ Umat[:, :20].conj().T
    e_proj = float(np.abs(Vs @ Vs.conj().T - Po).max())
    e_orth = float(np.abs(basis.conj() @ basis.T - np.eye(len(basis))).max())
    e_eig = float(np.abs(ev[:21] - np.sort(vals)[::-1][:21]).max() / 100.0)
    V = basis[:rs + 1].T
    resid = np.linalg.norm(g @ V - V * ev[:rs + 1], axis=0).max() / ev[0]
    gap = 1.0 - noise
    bound = np.sqrt(rs + 1) * 1e-10 * ev[0] / gap
    report("nullspace repeated", r=rs, iters=int(counts[2]), err_eig=e_eig,
           err_proj=e_proj, err_orth=e_orth, resid=float(resid), proj_bound=float(bound))
    assert counts[3] == 1 and rs == 20
    assert e_eig <= 1e-12 and e_orth <= 1e-10
    assert resid <= 1e-10 * (1 + 1e-6) and e_proj <= bound


# ------------------------------------------------------------------ G(x)


PRECISIONS = {0: "fp32", 1: "split_f16", 2: "split_bf16"}


@pytest.mark.parametrize("prec", list(PRECISIONS))
@pytest.mark.parametrize("name", WLALL)
def test_gx(name, prec):
    """G(x) against the oracle for each arithmetic of the contraction over
    the signal vectors (FP32, or FP16 / BF16 matrix cores with split
    operands and FP32 accumulation); the error vs FP64 is printed."""
    w, _ = scan_inputs(name)
    lam, lags, _, _, sp = oracle_gram_split(name)
    est = estimator(name, precision=prec)
    b = est.block
    basis = np.ascontiguousarray(sp.vectors[:, :b].T)
    counts = np.array([sp.r_signal, b, 0, 1], dtype=np.int32)
    G = est.gx(cuda(basis), cuda(counts)).cpu().numpy()
    Kn = lagkernel.lag_kernel_from_filters(sp.null, lam, lags, w.Q)
    if w.D == 2:
        idx = np.arange(int(np.prod(w.grid_lr)))
        pts = ogx.grid_points(w.grid_lr)
    else:
        idx, pts = sampled_points(w.grid_lr, 600, 77)
    Go = packed_upper(ogx.gx_from_lag_kernel(Kn, lags, pts))
    err = float(np.abs(G[:, idx] - Go).max() / len(lam))
    report(f"gx {name} {PRECISIONS[prec]}", err=err, sampled=len(idx))
    assert err <= 1e-5


# ------------------------------------------------------------------ per-voxel eigenvectors


def _eig_compare(est, G, Q, bound, tag, n_iter=10, tol=0.0):
    import paper_2302_13431_amd as P
    G32 = G.astype(np.complex64)
    Gw = G32.astype(np.complex128)
    opts = P.make_opts(power_iters=n_iter, tol=tol)
    maps, lam, it = est.eig(cuda(packed_upper(G32)), N=len(G), opts=opts, Q=Q, bound=bound)
    maps, lam, it = maps.cpu().numpy(), lam.cpu().numpy(), it.cpu().numpy()
    c, lo, _, ito = oeig.power_iteration(Gw, bound, n_iter, tol if tol > 0 else None,
                                         max_iter=n_iter)
    # the start index is a floating-point decision: compare only where the
    # two largest diagonal entries of Gs are separated by more than rounding
    d = np.sort(np.real(np.einsum("xqq->xq", Gw)), axis=1)
    clear = (d[:, 1] - d[:, 0]) > 1e-5 * bound if Q > 1 else np.ones(len(G), bool)
    e = map_error(c, maps.T, axis=1)
    e_lam = float(np.abs(lam - lo).max() / bound)
    report(tag, err_map=float(e[clear].max()), err_lam=e_lam, ambiguous=int((~clear).sum()))
    assert float(e[clear].max()) <= 1e-4
    assert e_lam <= 1e-5
    assert np.allclose(np.linalg.norm(maps, axis=0), 1.0, atol=1e-5)
    if tol > 0:
        assert np.mean(it == ito) > 0.99 and np.all(np.abs(it - ito) <= 1)
    else:
        assert np.all(it == n_iter)


@pytest.mark.parametrize("name", WL2D)
def test_eig_on_oracle_field(name):
    ref = oracle_full(name)
    w = workloads.ALL[name]
    _eig_compare(estimator(name), ref.G, w.Q, float(len(ref.lam)), "eig " + name)


@pytest.mark.parametrize("Q,N", [(2, 333), (3, 1000), (5, 257), (8, 4099), (15, 1031),
                                 (16, 2048), (32, 1537)])
def test_eig_random_fields(Q, N):
    rng = np.random.default_rng(100 + Q)
    bound = 30.0
    U = np.linalg.qr(rng.standard_normal((N, Q, Q)) + 1j * rng.standard_normal((N, Q, Q)))[0]
    w = np.sort(rng.uniform(0.2, 1.0, size=(N, Q)), axis=1) * bound
    w[:, 0] = rng.uniform(0.0, 0.05, size=N) * bound
    G = np.einsum("xpk,xk,xqk->xpq", U, w, U.conj())
    est = estimator("2d_64x64_q8_acs24_r3")
    _eig_compare(est, G, Q, bound, f"eig random Q={Q} N={N}")
    _eig_compare(est, G, Q, bound, f"eig random tol Q={Q} N={N}", n_iter=60, tol=1e-3)


def test_eig_empty():
    import paper_2302_13431_amd as P
    est = estimator("2d_64x64_q8_acs24_r3")
    dummy = torch.zeros(1, dtype=torch.complex64, device="cuda")
    maps = torch.zeros(1, dtype=torch.complex64, device="cuda")
    P.pisco_eig(est.h, 8, 0, 29.0, est.opts, dummy, maps)
    torch.cuda.synchronize()


@pytest.mark.parametrize("name", WL2D)
@pytest.mark.parametrize("tol", [0.0, 1e-4])
def test_eig_fp64_rayleigh_check(name, tol):
    """FP64 Rayleigh quotient and residual of the FP32 maps (Sec. IV-E check)
    against the oracle's definition on the same vectors and the same (FP32)
    matrices, to 1e-12 |Lambda|; in tolerance mode every voxel that stopped
    before the cap meets the tolerance in FP64 too (up to FP32 rounding of
    the stopping test)."""
    import paper_2302_13431_amd as P
    ref = oracle_full(name)
    w = workloads.ALL[name]
    bound = float(len(ref.lam))
    G32 = ref.G.astype(np.complex64)
    est = estimator(name)
    opts = P.make_opts(power_iters=10 if tol == 0 else 100, tol=tol)
    maps, lam, it, lam64, res64 = est.eig_checked(cuda(packed_upper(G32)), opts=opts)
    maps, lam, it = maps.cpu().numpy(), lam.cpu().numpy(), it.cpu().numpy()
    lam64, res64 = lam64.cpu().numpy(), res64.cpu().numpy()
    lo, ro = oeig.rayleigh(G32.astype(np.complex128), maps.T)
    e_l = float(np.abs(lam64 - lo).max() / bound)
    e_r = float(np.abs(res64 - ro).max() / bound)
    _, _, r_pi, _ = oeig.power_iteration(ref.G, bound, 10)
    report(f"eig fp64 check {name} tol={tol}", err_lam64=e_l, err_res64=e_r,
           res_max=float(res64.max() / bound), oracle_pi_res_max=float(r_pi.max() / bound),
           lam32_vs_64=float(np.abs(lam - lam64).max() / bound))
    assert e_l <= 1e-12 and e_r <= 1e-12
    assert float(np.abs(lam - lam64).max() / bound) <= 1e-5
    if tol > 0:
        stopped = it < 100
        assert stopped.mean() > 0.99
        assert np.all(res64[stopped] <= tol * bound * (1 + 1e-2) + 1e-5 * bound)


# ------------------------------------------------------------------ phase + interpolation


@pytest.mark.parametrize("name", WLALL)
@pytest.mark.parametrize("rule", [0, 1])
def test_maps(name, rule):
    ref = oracle_full(name)
    w, acs = scan_inputs(name)
    est = estimator(name, phase_rule=rule)
    c32 = ref.c_lr.astype(np.complex64)
    out = est.maps(cuda(acs), cuda(c32.reshape(w.Q, -1))).cpu().numpy()
    cw = c32.astype(np.complex128)
    if rule == 0:
        cref, _ = omaps.phase_reference(cw, ref.rho_lr)
        mask_lr = lowres_mask(cw, ref.rho_lr, None)
    else:
        cref = omaps.coil_reference(cw)
        mag = np.abs(cw[0])
        from scipy.ndimage import binary_erosion
        mask_lr = binary_erosion(mag >= 1e-3 * mag.max(), iterations=1)
    o = omaps.normalize_rss(omaps.interpolate(cref, w.grid))
    e = map_error(o, out)
    mo = output_mask(mask_lr, w.grid)
    report(f"maps {name} rule={rule}", err_mask=float(e[mo].max()), err_all=float(e.max()),
           mask_frac=float(mo.mean()), abs_mask=float(np.abs(out - o)[:, mo].max()))
    assert float(e[mo].max()) <= 1e-4
    rss = np.sqrt(np.sum(np.abs(out) ** 2, axis=0))
    assert np.allclose(rss, 1.0, atol=1e-5)


# ------------------------------------------------------------------ end to end


PRODUCTS = {1: "dense", 2: "structured"}


@pytest.mark.parametrize("name", WLALL)
@pytest.mark.parametrize("prec", list(PRECISIONS))
@pytest.mark.parametrize("product", list(PRODUCTS))
def test_end_to_end(name, prec, product):
    """The whole path against the oracle, with the nullspace's Gram products
    either on the explicit Gram or through its correlation structure (the
    Gram never formed)."""
    ref = oracle_full(name)
    w, acs = scan_inputs(name)
    est = estimator(name, precision=prec, product=product)
    out, lam = est.estimate(cuda(acs))
    out, lam = out.cpu().numpy(), lam.cpu().numpy()
    bound = float(len(ref.lam))
    e_lam = float(np.abs(lam - ref.lam_min).max() / bound)
    mask_lr = lowres_mask(ref.c_lr, ref.rho_lr, None)
    mo = output_mask(mask_lr, w.grid)
    e = map_error(ref.maps, out)
    report(f"e2e {name} {PRECISIONS[prec]} {PRODUCTS[product]}", err_lam=e_lam,
           err_map_mask=float(e[mo].max()), err_map_p99=float(np.percentile(e, 99)),
           err_map_all=float(e.max()))
    assert est.status() == 0
    assert e_lam <= 1e-5
    assert float(e[mo].max()) <= 1e-4


def test_end_to_end_ragged():
    """Odd ACS, non-integer radius, non-square grids, Q = 5."""
    import paper_2302_13431_amd as P
    from oracle import pipeline as opipe
    sc = generator.make_scan(55, (50, 61), 5, (23, 25), 4, 40.0, keep_kspace=False)
    acs = generator.as_device_input(sc.acs)
    lr, out_grid, radius = (21, 27), (50, 61), 2.5
    ref = opipe.estimate(acs.astype(np.complex128), radius, lr, out_grid)
    est = P.Estimator(5, (23, 25), radius, lr, out_grid, block=32)
    out, lam = est.estimate(cuda(acs))
    out, lam = out.cpu().numpy(), lam.cpu().numpy()
    mo = output_mask(lowres_mask(ref.c_lr, ref.rho_lr, None), out_grid)
    e = map_error(ref.maps, out)
    e_lam = float(np.abs(lam - ref.lam_min).max() / len(ref.lam))
    report("e2e ragged", r_s=ref.split.r_signal, err_lam=e_lam, err_map=float(e[mo].max()))
    assert e_lam <= 1e-5 and float(e[mo].max()) <= 1e-4


@pytest.mark.parametrize("product", list(PRODUCTS))
def test_end_to_end_small_3d(product):
    """Odd extents in every dimension, radius 2 (a 5^3 box, 9^3 frequency
    grid for the structured products)."""
    import paper_2302_13431_amd as P
    from oracle import pipeline as opipe
    sc = generator.make_scan(66, (24, 28, 32), 4, (12, 12, 12), 4, 40.0, keep_kspace=False)
    acs = generator.as_device_input(sc.acs)
    lr, out_grid, radius = (16, 18, 20), (24, 28, 32), 2.0
    ref = opipe.estimate(acs.astype(np.complex128), radius, lr, out_grid)
    est = P.Estimator(4, (12, 12, 12), radius, lr, out_grid, block=64, product=product)
    out, lam = est.estimate(cuda(acs))
    out, lam = out.cpu().numpy(), lam.cpu().numpy()
    mo = output_mask(lowres_mask(ref.c_lr, ref.rho_lr, None), out_grid)
    e = map_error(ref.maps, out)
    e_lam = float(np.abs(lam - ref.lam_min).max() / len(ref.lam))
    report(f"e2e small 3d {PRODUCTS[product]}", r_s=ref.split.r_signal, err_lam=e_lam,
           err_map=float(e[mo].max()))
    assert est.status() == 0
    assert e_lam <= 1e-5 and float(e[mo].max()) <= 1e-4


# ------------------------------------------------------------------ failure handling


def test_nonfinite_input_is_flagged():
    import paper_2302_13431_amd as P
    w, acs = scan_inputs("2d_64x64_q8_acs24_r3")
    bad = acs.copy()
    bad[0, 3, 4] = np.nan
    est = estimator("2d_64x64_q8_acs24_r3")
    est.estimate(cuda(bad))
    assert est.status() & P._lib.FLAG_NONFINITE


def test_zero_data_is_flagged():
    import paper_2302_13431_amd as P
    w, acs = scan_inputs("2d_64x64_q8_acs24_r3")
    est = estimator("2d_64x64_q8_acs24_r3")
    out, lam = est.estimate(cuda(np.zeros_like(acs)))
    assert est.status() & P._lib.FLAG_ZERO_DATA
    assert torch.isfinite(torch.view_as_real(out)).all()


def test_block_too_small_is_flagged():
    """A block narrower than the signal rank plus its margin (forced from the
    host: block 32 against the 71 signal eigenvalues of the 256^2 scan)."""
    import paper_2302_13431_amd as P
    name = "2d_256x256_q32_acs32_r5"
    _, _, _, g32, sp = oracle_gram_split(name)
    assert sp.r_signal > 32
    est = estimator(name, block=32)
    ev, basis, counts = est.nullspace(cuda(g32))
    flags = est.status()
    report("block too small", flags=flags, counts=str(counts.cpu().numpy().tolist()))
    assert flags & P._lib.FLAG_BLOCK_TOO_SMALL


def test_not_converged_is_flagged():
    """An iteration cap the schedule cannot meet (forced from the host: at
    most three products, before the first Rayleigh-Ritz step is due)."""
    import paper_2302_13431_amd as P
    name = "2d_256x256_q32_acs32_r5"
    _, _, _, g32, _ = oracle_gram_split(name)
    est = estimator(name, max_subspace_iters=3)
    ev, basis, counts = est.nullspace(cuda(g32))
    counts = counts.cpu().numpy()
    flags = est.status()
    report("not converged", flags=flags, counts=str(counts.tolist()))
    assert flags & P._lib.FLAG_NOT_CONVERGED
    assert counts[3] == 0


@pytest.mark.parametrize("name", WLALL)
def test_device_schedule_matches_oracle(name):
    """The device-resident nullspace schedule (nothing read back on the host)
    against the oracle, stage and end to end."""
    import paper_2302_13431_amd as P
    _, _, _, g32, sp = oracle_gram_split(name)
    est = estimator(name, schedule=P._lib.SCHED_DEVICE)
    ev, basis, counts = est.nullspace(cuda(g32))
    ev, basis, counts = ev.cpu().numpy(), basis.cpu().numpy(), counts.cpu().numpy()
    rs = int(counts[0])
    Vs = basis[:rs].T
    e_proj = float(np.abs(Vs @ Vs.conj().T - sp.signal @ sp.signal.conj().T).max())
    e_eig = float(np.abs(ev[:rs + 1] - sp.eigvals[:rs + 1]).max() / sp.eigvals[0])
    ref = oracle_full(name)
    w, acs = scan_inputs(name)
    out, lam = est.estimate(cuda(acs))
    out, lam = out.cpu().numpy(), lam.cpu().numpy()
    mo = output_mask(lowres_mask(ref.c_lr, ref.rho_lr, None), w.grid)
    e = map_error(ref.maps, out)
    e_lam = float(np.abs(lam - ref.lam_min).max() / len(ref.lam))
    report("device schedule " + name, products=int(counts[2]), r=rs, err_eig=e_eig,
           err_proj=e_proj, err_lam=e_lam, err_map=float(e[mo].max()))
    assert counts[3] == 1 and rs == sp.r_signal
    assert e_eig <= 1e-5 and e_proj <= 1e-7
    assert e_lam <= 1e-5 and float(e[mo].max()) <= 1e-4
    assert est.status() == 0


def test_estimate_captured_on_fresh_handle():
    """pisco_estimate recorded into a HIP graph on a handle that has never
    run (default schedule: device-resident under capture; tables built in
    the workspace by the captured call itself), replayed three times with
    eager work in between, each replay against the oracle."""
    import paper_2302_13431_amd as P
    name = "2d_256x256_q32_acs32_r5"
    ref = oracle_full(name)
    w, acs = scan_inputs(name)
    est = estimator(name)
    x = cuda(acs)
    out = torch.empty((w.Q,) + tuple(w.grid), dtype=torch.complex64, device="cuda")
    lam = torch.empty((int(np.prod(w.grid_lr)),), dtype=torch.float32, device="cuda")
    size = P._lib.pisco_workspace_size(est.prob, est.opts, P._lib.STAGE_ALL)
    raw = torch.empty(size + 256, dtype=torch.uint8, device="cuda")
    ws = raw[(-raw.data_ptr()) % 256:]
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    est.h.set_stream(s)
    try:
        with torch.cuda.graph(g, stream=s):
            P.pisco_estimate(est.h, est.prob, est.opts, x, out, lam, ws)
    finally:
        est.h.set_stream(None)
    mo = output_mask(lowres_mask(ref.c_lr, ref.rho_lr, None), w.grid)
    bound = float(len(ref.lam))
    for rep in range(3):
        out.zero_()
        lam.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        o, l = out.cpu().numpy(), lam.cpu().numpy()
        e = map_error(ref.maps, o)
        e_lam = float(np.abs(l - ref.lam_min).max() / bound)
        report(f"captured estimate replay {rep}", err_lam=e_lam, err_map=float(e[mo].max()))
        assert est.status() == 0
        assert e_lam <= 1e-5 and float(e[mo].max()) <= 1e-4


def test_workspace_too_small_is_rejected():
    import paper_2302_13431_amd as P
    w, acs = scan_inputs("2d_64x64_q8_acs24_r3")
    est = estimator("2d_64x64_q8_acs24_r3")
    tiny = torch.empty(256, dtype=torch.uint8, device="cuda")
    gram = torch.empty((est.n, est.n), dtype=torch.complex64, device="cuda")
    with pytest.raises(P.PiscoError) as ex:
        P.pisco_gram(est.h, est.prob, cuda(acs), gram, tiny)
    assert ex.value.status == 2


def test_binding_refuses_undersized_buffers():
    """The library takes raw device pointers, so the binding checks every
    buffer against the bytes the call will touch and raises before any
    launch: a basis argument that is really the eigenvalue vector, a G field
    for fewer voxels, a CPU tensor, a non-contiguous output."""
    name = "2d_64x64_q8_acs24_r3"
    w, acs = scan_inputs(name)
    est = estimator(name)
    ev = torch.zeros(est.block, dtype=torch.float64, device="cuda")
    counts = torch.zeros(4, dtype=torch.int32, device="cuda")
    with pytest.raises(ValueError, match="basis"):
        est.gx(ev, counts)
    G_small = torch.zeros((est.P, est.Nlr - 1), dtype=torch.complex64, device="cuda")
    for call in (lambda: est.eig(G_small), lambda: est.eig_sets(G_small),
                 lambda: est.espirit_operator(G_small)):
        with pytest.raises(ValueError, match="G"):
            call()
    with pytest.raises(ValueError, match="CUDA"):
        est.gram(torch.from_numpy(acs))
    out = torch.empty((w.Q,) + tuple(w.grid)[::-1], dtype=torch.complex64,
                      device="cuda").transpose(1, 2)
    with pytest.raises(ValueError, match="contiguous"):
        est.estimate(cuda(acs), out)
    assert est.status() == 0
