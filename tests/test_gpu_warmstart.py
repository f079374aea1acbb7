"""Learned warm start on the GPU: forward pass and gradients against the FP64
oracle (oracle/mlp.py) on the same weights and inputs, the start-vector
semantics of pisco_eig_from, and what a network trained by the library's
own kernels gains over the plain start.

Tolerances: inference runs in FP16 (weights and activations) with FP32
accumulation, so its outputs carry relative errors of order 1e-3 against
FP64 on the same FP16-rounded weights (check: 1e-2 per entry).  Training
carries features, activations and per-voxel gradients as FP16 pairs (FP32
values) and sums the weight gradients in FP32, so the gradient of the summed
loss agrees with the FP64 oracle on the same FP16 weights to 2e-3 per
parameter block in the 2-norm.  Adam is checked against the oracle's update
over several steps on the library's own gradients."""
import numpy as np
import pytest

from oracle import mlp
from synth import generator, workloads

from .gpu_common import oracle_full

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2302_13431_amd  # noqa: F401


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def report(tag, **vals):
    print(f"[{tag}] " + " ".join(f"{k}={v:.3e}" if isinstance(v, float) else f"{k}={v}"
                                 for k, v in vals.items()), flush=True)


def packed(G):
    """[N, Q, Q] Hermitian -> packed upper planes [P][N] (complex64)."""
    N, Q, _ = G.shape
    rows = [G[:, p, q] for p in range(Q) for q in range(p, Q)]
    return np.ascontiguousarray(np.stack(rows).astype(np.complex64))


def _case(seed=3, N=600, scale_out=1.0):
    """Oracle G field of the 64x64, 8-channel workload, seeded neighbour and
    target vectors and seeded weights (FP16-rounded, both sides use them)."""
    ref = oracle_full("2d_64x64_q8_acs24_r3")
    G = ref.G[:N]
    Q = G.shape[1]
    bound = float(len(ref.lam))
    rng = np.random.default_rng(seed)
    nb = mlp.gauge_fix(rng.standard_normal((N, Q)) + 1j * rng.standard_normal((N, Q)))
    nb /= np.linalg.norm(nb, axis=1, keepdims=True)
    tgt = rng.standard_normal((N, Q)) + 1j * rng.standard_normal((N, Q))
    tgt /= np.linalg.norm(tgt, axis=1, keepdims=True)
    din, h, dout = mlp.dims(Q)
    parts = [rng.uniform(-1, 1, h * din) * np.sqrt(6 / din), 0.1 * rng.standard_normal(h),
             rng.uniform(-1, 1, h * h) * np.sqrt(6 / h), 0.1 * rng.standard_normal(h),
             scale_out * rng.uniform(-1, 1, dout * h) * np.sqrt(6 / h),
             0.1 * rng.standard_normal(dout)]
    theta16 = np.concatenate(parts).astype(np.float16)
    return G, nb, tgt, bound, Q, theta16


def _ws_with(theta16, Q):
    import paper_2302_13431_amd as P
    ws = P.WarmStart(Q)
    assert ws.count == len(theta16) == mlp.param_count(Q)
    ws.w16.copy_(cuda(theta16))
    ws.master.copy_(cuda(theta16.astype(np.float32)))
    return ws


def test_ws_forward_matches_oracle():
    G, nb, tgt, bound, Q, th16 = _case()
    ws = _ws_with(th16, Q)
    init = ws.forward(cuda(packed(G)), cuda(nb.T.astype(np.complex64)), bound).cpu().numpy().T
    theta = th16.astype(np.float64)
    c_hat, _ = mlp.forward(theta, mlp.features(G, nb, bound), nb, Q)
    ref = c_hat / np.linalg.norm(c_hat, axis=1, keepdims=True)
    err = float(np.abs(init - ref).max())
    report("ws forward", err=err, y_scale=float(np.abs(c_hat - nb).mean()))
    assert err <= 1e-2


def test_ws_gradient_matches_oracle():
    G, nb, tgt, bound, Q, th16 = _case(seed=4)
    ws = _ws_with(th16, Q)
    loss, grad = ws.gradient(cuda(packed(G)), cuda(nb.T.astype(np.complex64)),
                             cuda(tgt.T.astype(np.complex64)), bound)
    loss, grad = float(loss.item()), grad.cpu().numpy().astype(np.float64)
    theta = th16.astype(np.float64)
    L0, gmean = mlp.batch_loss_and_grad(theta, G, nb, tgt, bound, Q)
    gsum = gmean * len(G)
    errs = []
    for name, a, b in zip(["W1", "b1", "W2", "b2", "W3", "b3"], mlp.unpack(grad, Q),
                          mlp.unpack(gsum, Q)):
        e = float(np.linalg.norm(a - b) / np.linalg.norm(b))
        errs.append(e)
        report("ws grad " + name, rel_err=e)
    report("ws loss", gpu=loss, oracle=L0)
    assert abs(loss - L0) <= 1e-4 * max(1.0, abs(L0))
    assert max(errs) <= 2e-3


def test_ws_adam_matches_oracle():
    """Five Adam steps on one batch: after each, the FP32 master weights and
    both moments equal the oracle's adam_step applied to the same gradients
    (the library's own, taken at the current weights before each step)."""
    G, nb, tgt, bound, Q, th16 = _case(seed=6)
    ws = _ws_with(th16, Q)
    Gd, nbd, td = cuda(packed(G)), cuda(nb.T.astype(np.complex64)), cuda(tgt.T.astype(np.complex64))
    theta = th16.astype(np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    lr = 1e-3
    n = len(G)
    for step in range(1, 6):
        _, grad = ws.gradient(Gd, nbd, td, bound)
        g = grad.cpu().numpy().astype(np.float64) / n
        theta, m, v = mlp.adam_step(theta, m, v, g, step, lr)
        ws.train_step(Gd, nbd, td, bound, lr)
        master = ws.master.cpu().numpy().astype(np.float64)
        ulp = np.spacing(np.abs(theta).astype(np.float32)).astype(np.float64)
        e_w = float(np.max(np.abs(master - theta) / (2 * step * ulp + step * 1e-5 * lr)))
        e_m = float(np.abs(ws.m.cpu().numpy() - m).max() / np.abs(m).max())
        e_v = float(np.abs(ws.v.cpu().numpy() - v).max() / np.abs(v).max())
        report(f"ws adam step {step}", w_over_bound=e_w, m_rel=e_m, v_rel=e_v)
        assert e_w <= 1.0 and e_m <= 1e-5 and e_v <= 1e-5
    assert np.array_equal(ws.w16.cpu().numpy(), ws.master.cpu().numpy().astype(np.float16))


def test_ws_adam_step():
    """One step from zero moments moves each weight by at most lr, opposite
    to the (mean) gradient wherever that gradient is not tiny."""
    G, nb, tgt, bound, Q, th16 = _case(seed=5)
    ws = _ws_with(th16, Q)
    Gd, nbd, td = cuda(packed(G)), cuda(nb.T.astype(np.complex64)), cuda(tgt.T.astype(np.complex64))
    _, grad = ws.gradient(Gd, nbd, td, bound)
    before = ws.master.clone()
    lr = 1e-3
    ws.train_step(Gd, nbd, td, bound, lr)
    d = (ws.master - before).cpu().numpy()
    g = grad.cpu().numpy()
    big = np.abs(g) > 1e-3 * np.abs(g).max()
    assert np.abs(d).max() <= lr * (1 + 1e-4)
    assert np.mean(np.sign(d[big]) == -np.sign(g[big])) > 0.999
    assert np.array_equal(ws.w16.cpu().numpy(), ws.master.cpu().numpy().astype(np.float16))


def test_eig_from_start_vectors():
    """From the exact eigenvector the iteration stops at once (tolerance
    mode); from zero vectors it falls back to the plain start."""
    import paper_2302_13431_amd as P
    ref = oracle_full("2d_64x64_q8_acs24_r3")
    w = workloads.ALL["2d_64x64_q8_acs24_r3"]
    G = ref.G
    N, Q = G.shape[0], G.shape[1]
    est = P.Estimator(w.Q, w.acs, w.radius, w.grid_lr, w.grid, block=64)
    Gd = cuda(packed(G))
    lam, V = np.linalg.eigh(G)
    exact = cuda(np.ascontiguousarray(V[:, :, 0].T.astype(np.complex64)))
    tol = P.make_opts(power_iters=500, tol=1e-4, block=64)
    _, _, it = est.eig_from(Gd, exact, tol)
    assert int(it.max().item()) <= 1
    zero = torch.zeros((Q, N), dtype=torch.complex64, device="cuda")
    m0, l0, i0 = est.eig(Gd, opts=tol)
    m1, l1, i1 = est.eig_from(Gd, zero, tol)
    assert torch.equal(m0, m1) and torch.equal(i0, i1)


def _scan_acs(seed):
    w = workloads.SMALL_2D
    sc = generator.make_scan(seed, w.grid, w.Q, w.acs, 6, w.snr_db, keep_kspace=False)
    return cuda(generator.as_device_input(sc.acs))


def test_warm_start_gain():
    """Train on the method's own eigenvectors of 8 seeded scans (64x64, 8
    channels), then on a held-out scan compare the power-iteration steps
    needed for ||G c - lambda c|| <= 1e-4 |Lambda| from the plain start and
    from the network's start, with the final residuals checked in FP64."""
    import paper_2302_13431_amd as P
    w = workloads.SMALL_2D
    est = P.Estimator(w.Q, w.acs, w.radius, w.grid_lr, w.grid, block=64)
    est_c = P.Estimator(w.Q, w.acs, w.radius, P.coarse_grid(w.grid_lr), w.grid, block=64)
    ws = P.WarmStart(w.Q, seed=7)
    from paper_2302_13431_amd.warmstart import LearnedSolver
    solver = LearnedSolver(est, est_c, ws)
    bound = float(est.nsup)
    tight = P.make_opts(power_iters=4000, tol=1e-6, block=64)
    data = []
    for seed in range(100, 108):
        G, Gc = solver.fields(_scan_acs(seed))
        nb = solver.neighbour(Gc)
        target, _, _ = est.eig(G, opts=tight)
        data.append((G, nb, target))
    losses = []
    for epoch in range(40):
        tot = 0.0
        for G, nb, target in data:
            tot += float(ws.train_step(G, nb, target, bound, 2e-3).item())
        losses.append(tot / len(data))
    G, Gc = solver.fields(_scan_acs(999))
    opts = P.make_opts(power_iters=4000, tol=1e-4, block=64)
    m_plain, l_plain, it_plain = est.eig(G, opts=opts)
    m_ws, l_ws, it_ws = solver.solve(G, Gc, opts)
    nb = solver.neighbour(Gc)
    _, _, it_nb = est.eig_from(G, nb, opts)
    # FP64 residuals of both results on the same G
    Gh = G.cpu().numpy().astype(np.complex128)
    Q = w.Q
    Gm = np.zeros((Gh.shape[1], Q, Q), complex)
    k = 0
    for p in range(Q):
        for q in range(p, Q):
            Gm[:, p, q] = Gh[k]
            Gm[:, q, p] = np.conj(Gh[k])
            k += 1

    def resid(m):
        c = m.cpu().numpy().T.astype(np.complex128)
        c /= np.linalg.norm(c, axis=1, keepdims=True)
        Gc_ = np.einsum("xpq,xq->xp", Gm, c)
        lam = np.real(np.sum(np.conj(c) * Gc_, axis=1))
        return np.linalg.norm(Gc_ - lam[:, None] * c, axis=1) / bound

    r_plain, r_ws = resid(m_plain), resid(m_ws)
    ip, iw, inb = (float(i.float().mean().item()) for i in (it_plain, it_ws, it_nb))
    report("ws gain", loss_first=losses[0], loss_last=losses[-1], iters_plain=ip,
           iters_neighbour=inb, iters_learned=iw, resid_plain_p99=float(np.percentile(r_plain, 99)),
           resid_learned_p99=float(np.percentile(r_ws, 99)))
    assert losses[-1] < losses[0]
    assert np.percentile(r_plain, 99) <= 2e-4 and np.percentile(r_ws, 99) <= 2e-4
    assert iw < ip
