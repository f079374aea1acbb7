"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point declared in include/pisco.h, and its host-only calls agree
with their definitions."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pisco.h")


def _lib():
    from paper_2302_13431_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        from paper_2302_13431_amd import build
        build.build()
    return L


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pisco_[a-z_]+)\s*\(", text)))


def test_header_declares_the_five_stages():
    names = declared_functions()
    for n in ("pisco_gram", "pisco_nullspace", "pisco_gx", "pisco_eig", "pisco_maps"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = _lib()
    lib = L.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_support_matches_definition():
    """Lambda = {n : ||n||_2 <= r}, lexicographic with x fastest; compared with
    a direct enumeration and with the oracle's (same ordering convention)."""
    L = _lib()
    from oracle import support as osup
    for D, r in [(2, 1.0), (2, 3.0), (2, 3.5), (2, 6.0), (3, 2.0), (3, 4.0), (3, 5.0)]:
        pts = L.pisco_support(D, r)
        if D == 2:
            assert all(p[0] == 0 for p in pts)
            got = np.array([p[1:] for p in pts])
        else:
            got = np.array(pts)
        ref = osup.kernel_support(D, r)
        assert np.array_equal(got, ref), (D, r)
    for D, r in [(2, 1.0), (2, 3.5), (3, 2.0), (3, 3.0)]:
        pts = L.pisco_support(D, r, L.SHAPE_RECTANGLE)
        got = np.array([p[1:] for p in pts]) if D == 2 else np.array(pts)
        assert np.array_equal(got, osup.kernel_support(D, r, "rectangle")), (D, r)


def test_problem_validation():
    L = _lib()
    ok = L.make_problem(2, 8, (24, 24), 3.0, (32, 32), (64, 64))
    assert L.pisco_workspace_size(ok, None, L.STAGE_GRAM) > 0
    bad = [
        L.make_problem(2, 1, (24, 24), 3.0, (32, 32), (64, 64)),     # Q < 2
        L.make_problem(2, 33, (24, 24), 3.0, (32, 32), (64, 64)),    # Q > 32
        L.make_problem(2, 8, (6, 6), 3.0, (32, 32), (64, 64)),       # ACS <= 2 tau
        L.make_problem(2, 8, (24, 24), 0.5, (32, 32), (64, 64)),     # radius < 1
        L.make_problem(2, 8, (24, 24), 3.0, (32, 32), (16, 64)),     # out < lr
        L.make_problem(4, 8, (24, 24), 3.0, (32, 32), (64, 64)),     # D
        L.make_problem(2, 8, (24, 24), 3.0, (32, 32), (64, 64), thresh=0.0),
        L.make_problem(2, 8, (300, 24), 3.0, (32, 32), (512, 64)),   # FFT > 256
    ]
    for p in bad:
        with pytest.raises(L.PiscoError) as ex:
            L.pisco_workspace_size(p, None, L.STAGE_GRAM)
        assert ex.value.status == 1


def test_null_handle_is_rejected_without_device_work():
    L = _lib()
    p = L.make_problem(2, 8, (24, 24), 3.0, (32, 32), (64, 64))
    lib = L.lib()
    assert lib.pisco_gram(None, p, None, None, None, 0) == 1
    assert lib.pisco_estimate(None, p, None, None, None, None, None, 0) == 1
    assert lib.pisco_destroy(None) == 1


def test_block_rules():
    L = _lib()
    p = L.make_problem(2, 32, (32, 32), 5.0, (56, 56), (256, 256))
    assert L.pisco_nullspace_block(p, None) == 96
    with pytest.raises(L.PiscoError):
        L.pisco_nullspace_block(p, L.make_opts(block=40))       # not a multiple of 32
    small = L.make_problem(2, 2, (12, 12), 1.0, (8, 8), (8, 8))  # n = 10 < 32
    with pytest.raises(L.PiscoError) as ex:
        L.pisco_nullspace_block(small, None)
    assert ex.value.status == 4


def test_workspace_sizes_cover_stage_buffers():
    L = _lib()
    p = L.make_problem(2, 32, (32, 32), 5.0, (56, 56), (256, 256))
    n, b = 32 * 81, 96
    total = L.pisco_workspace_size(p, None, L.STAGE_ALL)
    # Gram (FP32) + basis (FP64) + G + low-res maps at least
    assert total >= n * n * 8 + b * n * 16 + 528 * 56 * 56 * 8 + 32 * 56 * 56 * 8
    assert L.pisco_workspace_size(p, None, L.STAGE_NULLSPACE) >= 2 * n * b * 16


def test_status_strings():
    L = _lib()
    for st in range(6):
        assert L.pisco_status_string(st)
