"""Host build of the Rayleigh-Ritz eigensolver's arithmetic (CPU): the
tridiagonal routines the device kernels use, on graded spectra, exact and
near clusters and the zero matrix, for block sizes 1 to 224; eigenvalue
error, residual and orthogonality bounds are checked by the program."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2302_13431_amd", "csrc")


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("tri") / "tridiag_check")
    subprocess.run([gxx, "-O2", "-std=c++17", "-I", CSRC,
                    os.path.join(HERE, "host", "tridiag_check.cpp"), "-o", out], check=True)
    return out


@pytest.mark.parametrize("b,mode", [(96, 0), (96, 1), (96, 2), (96, 3), (224, 0), (224, 1),
                                    (5, 1), (1, 0), (2, 2), (33, 3)])
def test_tridiagonal_eigensolver(exe, b, mode):
    r = subprocess.run([exe, str(b), str(mode)], capture_output=True, text=True, timeout=120)
    print(r.stdout.strip())
    assert r.returncode == 0, r.stdout
