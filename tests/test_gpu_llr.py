"""Many small partial SVDs (pisco_llr_svd: locally low-rank models, Sec. I
and Sec. V) against the oracle's per-patch numpy SVD.

Patches of 8 x 8 pixels (m = 64) with Q columns, a singular spectrum
0.8^k up to the rank and a drop by 20 after it (a locally low-rank patch
plus a weaker remainder), plus noise; the Gram route resolves sigma_k to
about eps sigma_1^2 / sigma_k, so singular values are compared relative to
sigma_1 (<= 1e-5); the FP32 Gram moves the right singular subspace by
about eps sigma_1^2 / (sigma_r^2 - sigma_{r+1}^2), so the subspace
projectors and the rank-r parts (relative to the patch norm) are held to
100 eps sigma_1^2 / (sigma_r^2 - sigma_{r+1}^2), at least 1e-5."""
import numpy as np
import pytest

from oracle import llr

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2302_13431_amd  # noqa: F401


def _patches(rng, B, Q, m, rank):
    Uo = np.linalg.qr(rng.standard_normal((B, m, Q)) + 1j * rng.standard_normal((B, m, Q)))[0]
    Vo = np.linalg.qr(rng.standard_normal((B, Q, Q)) + 1j * rng.standard_normal((B, Q, Q)))[0]
    k = np.arange(Q)
    sig = np.where(k < rank, 0.8 ** k, 0.05 * 0.8 ** rank * 0.7 ** (k - rank))
    sig = sig * rng.uniform(0.5, 2.0, (B, 1))
    M = np.einsum("bik,bk,bqk->biq", Uo, sig, Vo.conj())
    M = M + 1e-4 * (rng.standard_normal(M.shape) + 1j * rng.standard_normal(M.shape))
    return np.ascontiguousarray(np.transpose(M, (0, 2, 1)).astype(np.complex64))


@pytest.mark.parametrize("Q,rank", [(8, 1), (8, 3), (16, 4), (32, 4), (32, 8)])
def test_llr_partial_svd(Q, rank):
    import paper_2302_13431_amd as P
    rng = np.random.default_rng(50 + Q + rank)
    B, m = 3000, 64
    X = _patches(rng, B, Q, m, rank)
    s_o, V_o, Xr_o = llr.partial_svd(X.astype(np.complex128), rank)
    h = P.Handle()
    Xd = torch.from_numpy(X).cuda()
    V = torch.empty((rank, Q, B), dtype=torch.complex64, device="cuda")
    Xr = torch.empty_like(Xd)
    sigma = P.pisco_llr_svd(h, Xd, rank, V, Xr)
    torch.cuda.synchronize()
    assert h.status() == 0
    s, V, Xr = sigma.cpu().numpy().T, V.cpu().numpy().transpose(2, 1, 0), Xr.cpu().numpy()
    e_s = float(np.max(np.abs(s - s_o) / s_o[:, :1]))
    Pg = np.einsum("bqk,bpk->bqp", V, V.conj())
    Po = np.einsum("bqk,bpk->bqp", V_o, V_o.conj())
    e_v = float(np.abs(Pg - Po).max())
    nrm = np.linalg.norm(X.reshape(B, -1), axis=1)
    e_x = float(np.max(np.linalg.norm((Xr - Xr_o).reshape(B, -1), axis=1) / nrm))
    print(f"[llr Q={Q} r={rank}] err_sigma={e_s:.2e} err_subspace={e_v:.2e} err_rank_part={e_x:.2e}",
          flush=True)
    s_all = np.linalg.svd(np.transpose(X.astype(np.complex128), (0, 2, 1)), compute_uv=False)
    gap = float(np.min((s_all[:, rank - 1] ** 2 - s_all[:, rank] ** 2) / s_all[:, 0] ** 2))
    tol = max(1e-5, 100 * np.finfo(np.float32).eps / 2 / gap)
    print(f"[llr Q={Q} r={rank}] relative Gram gap {gap:.3f}, subspace tolerance {tol:.1e}",
          flush=True)
    assert e_s <= 1e-5 and e_x <= tol and e_v <= tol
