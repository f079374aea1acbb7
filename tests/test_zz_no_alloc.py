"""pisco_gram_static (the Gram for callers that cannot allocate: the
library's static per-device scratch instead of a workspace) against
pisco_gram with a caller workspace: two calls in a row, the second on a
smaller problem, bit-identical results (same kernels, same order); a
problem beyond the scratch limit is refused before any launch."""
import numpy as np
import pytest

from synth import workloads

from .gpu_common import scan_inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2302_13431_amd  # noqa: F401


def _gram_pair(name):
    import paper_2302_13431_amd as P
    w, acs = scan_inputs(name)
    est = P.Estimator(w.Q, w.acs, w.radius, w.grid_lr, w.grid)
    x = torch.from_numpy(acs).cuda()
    ref = est.gram(x)
    out = torch.full_like(ref, float("nan"))
    need, limit = P.pisco_gram_static_bytes(est.prob)
    P.pisco_gram_static(est.h, est.prob, x, out)
    torch.cuda.synchronize()
    assert est.status() == 0
    print(f"[no-alloc gram {name}] scratch {need} of {limit} bytes", flush=True)
    return ref.cpu().numpy(), out.cpu().numpy()


def test_static_gram_matches_workspace_gram_twice():
    # larger problem first, then a smaller one in the same (reused) scratch
    for name in ("2d_256x256_q32_acs32_r5", "2d_64x64_q8_acs24_r3"):
        ref, out = _gram_pair(name)
        assert np.array_equal(ref, out), name


def test_static_gram_refuses_problem_beyond_limit():
    import paper_2302_13431_amd as P
    w = workloads.APP_3D
    prob = P.make_problem(w.D, w.Q, w.acs, w.radius, w.grid_lr, w.grid)
    need, limit = P.pisco_gram_static_bytes(prob)
    assert need > limit
    h = P.Handle()
    dummy = torch.zeros(1, dtype=torch.complex64, device="cuda")
    with pytest.raises(P.PiscoError) as ex:
        P.pisco_gram_static(h, prob, dummy, dummy)
    assert ex.value.status == 4
