"""Gram variants on the GPU against the oracle: the rectangular support of
Sec. III-C and the masked Gram C_valid^H C_valid (rows of C with no
implicit zeros, the form Sec. IV-A's correlation neglects), each as a stage
and end to end (the ablations behind the paper's Figs. 6 and 7)."""
import functools

import numpy as np
import pytest

from oracle import calib, pipeline as opipe, support
from oracle.metrics import map_error
from synth import workloads

from .gpu_common import lowres_mask, output_mask, scan_inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SHAPES = {0: "ellipsoid", 1: "rectangle"}
ROWS = {0: "full", 1: "valid"}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2302_13431_amd  # noqa: F401


def _est(name, shape, rows, **kw):
    import paper_2302_13431_amd as P
    w = workloads.ALL[name]
    return P.Estimator(w.Q, w.acs, w.radius, w.grid_lr, w.grid, shape=shape, gram_rows=rows, **kw)


@functools.lru_cache(maxsize=None)
def _oracle(name, shape, rows):
    w, acs = scan_inputs(name)
    return opipe.estimate(acs.astype(np.complex128), w.radius, w.grid_lr, w.grid,
                          shape=SHAPES[shape], rows=ROWS[rows])


@pytest.mark.parametrize("name", ["2d_64x64_q8_acs24_r3", "2d_256x256_q32_acs32_r5"])
@pytest.mark.parametrize("shape,rows", [(1, 0), (0, 1), (1, 1)])
def test_gram_variant(name, shape, rows):
    w, acs = scan_inputs(name)
    lam = support.kernel_support(w.D, w.radius, SHAPES[shape])
    a = acs.astype(np.complex128)
    if rows == 1:
        C = calib.calibration_matrix(a, lam, rows="valid")
        ref = C.conj().T @ C
    else:
        lags = support.difference_set(lam)
        ref = calib.gram_from_lags(calib.correlation_lags(a, lags), lam, lags)
    est = _est(name, shape, rows)
    g = est.gram(torch.from_numpy(acs).cuda()).cpu().numpy().astype(np.complex128)
    e_max = float(np.abs(g - ref).max() / np.abs(ref).max())
    e_fro = float(np.linalg.norm(g - ref) / np.linalg.norm(ref))
    print(f"[gram {name} {SHAPES[shape]} {ROWS[rows]}] n={len(ref)} err_max={e_max:.2e} "
          f"err_fro={e_fro:.2e}", flush=True)
    assert np.array_equal(g, g.conj().T)
    assert e_max <= 1e-5 and e_fro <= 1e-5
    assert est.status() == 0


@pytest.mark.parametrize("name", ["2d_64x64_q8_acs24_r3", "2d_256x256_q32_acs32_r5"])
@pytest.mark.parametrize("shape,rows", [(1, 0), (0, 1), (1, 1)])
def test_end_to_end_variant(name, shape, rows):
    ref = _oracle(name, shape, rows)
    w, acs = scan_inputs(name)
    est = _est(name, shape, rows, block=(ref.split.r_signal + 16 + 31) // 32 * 32 + 32)
    out, lam = est.estimate(torch.from_numpy(acs).cuda())
    out, lam = out.cpu().numpy(), lam.cpu().numpy()
    bound = float(len(ref.lam))
    e_lam = float(np.abs(lam - ref.lam_min).max() / bound)
    mo = output_mask(lowres_mask(ref.c_lr, ref.rho_lr, None), w.grid)
    e = map_error(ref.maps, out)
    print(f"[e2e {name} {SHAPES[shape]} {ROWS[rows]}] |Lambda|={len(ref.lam)} "
          f"r_s={ref.split.r_signal} block={est.block} err_lam={e_lam:.2e} "
          f"err_map={e[mo].max():.2e}", flush=True)
    assert est.status() == 0
    assert e_lam <= 1e-5 and float(e[mo].max()) <= 1e-4
