"""Host FP64 linear algebra of the library (eigenpairs, SVD, complex solve),
built from the library sources into a test shim with g++ and checked against
NumPy/LAPACK and against residual identities."""

import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

from pins import match_eigs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1805_05821_amd", "csrc")
EPS = 2.0 ** -52


@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("shim") / "libhostla_shim.so")
    cmd = [gxx, "-O2", "-std=c++17", "-shared", "-fPIC", f"-I{CSRC}",
           os.path.join(ROOT, "tests", "native", "hostla_shim.cpp"), os.path.join(CSRC, "hostla.cpp"), "-o", out]
    subprocess.run(cmd, check=True)
    lib = ctypes.CDLL(out)
    for f in (lib.shim_eig, lib.shim_svd, lib.shim_solve):
        f.restype = ctypes.c_int
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def eig(lib, A):
    m = A.shape[0]
    Af = np.asfortranarray(A, dtype=np.float64)
    lre, lim = np.zeros(m), np.zeros(m)
    zre, zim = np.zeros((m, m), order="F"), np.zeros((m, m), order="F")
    isr = np.zeros(m, dtype=np.int32)
    rc = lib.shim_eig(m, _p(Af), _p(lre), _p(lim), _p(zre), _p(zim), _p(isr))
    assert rc == 0
    return lre + 1j * lim, zre + 1j * zim, isr


def _check_eig(lib, A, tol_res=1e3):
    lam, Z, isr = eig(lib, A)
    m = A.shape[0]
    nA = max(np.linalg.norm(A, 2), 1e-300)
    R = A @ Z - Z * lam[None, :]
    res = np.linalg.norm(R, axis=0).max() / nA
    assert res <= tol_res * m * EPS, res
    assert np.allclose(np.linalg.norm(Z, axis=0), 1.0, atol=1e-12)
    assert np.all(lam[isr == 1].imag == 0.0)
    # pairs come as (re, +im), (re, -im)
    for i in range(m - 1):
        if isr[i] == 0 and lam[i].imag > 0:
            assert lam[i + 1] == np.conj(lam[i])
    ref = np.linalg.eigvals(A)
    return lam, ref


@pytest.mark.parametrize("m", [1, 2, 3, 5, 17, 64, 150])
def test_eig_random(shim, m):
    rng = np.random.default_rng(m)
    A = rng.standard_normal((m, m))
    lam, ref = _check_eig(shim, A)
    assert match_eigs(lam, ref) <= 1e-8 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("m", [4, 40, 300])
def test_eig_hessenberg_projected(shim, m):
    """Upper Hessenberg with positive subdiagonal, the shape of H_m."""
    rng = np.random.default_rng(100 + m)
    H = np.triu(rng.standard_normal((m, m)), -1)
    H[np.arange(1, m), np.arange(m - 1)] = np.abs(H[np.arange(1, m), np.arange(m - 1)]) + 0.1
    lam, ref = _check_eig(shim, H)
    assert match_eigs(lam, ref) <= 1e-7


def test_eig_special(shim):
    # diagonal, triangular, rotation (pure imaginary pair), zero, defective Jordan block
    _check_eig(shim, np.diag([3.0, -1.0, 2.0, 2.0]))
    _check_eig(shim, np.triu(np.arange(1.0, 26.0).reshape(5, 5)))
    lam, _ = _check_eig(shim, np.array([[0.0, -1.0], [1.0, 0.0]]))
    assert np.allclose(sorted(lam.imag), [-1, 1])
    lam, _ = _check_eig(shim, np.zeros((3, 3)))
    assert np.all(lam == 0)
    J = np.array([[2.0, 1.0, 0.0], [0.0, 2.0, 1.0], [0.0, 0.0, 2.0]])
    lam, Z, _ = eig(shim, J)
    assert np.allclose(lam, 2.0, atol=1e-5)
    # a real map with known complex spectrum (companion of a known polynomial)
    roots = np.array([0.9 * np.exp(0.3j), 0.9 * np.exp(-0.3j), 0.5, -0.7, 0.2 + 0.6j, 0.2 - 0.6j])
    c = np.poly(roots).real
    C = np.zeros((6, 6))
    C[0, :] = -c[1:]
    C[np.arange(1, 6), np.arange(5)] = 1.0
    lam, _ = _check_eig(shim, C)
    assert match_eigs(lam, roots) <= 1e-8


def test_svd_left(shim):
    rng = np.random.default_rng(7)
    for m in (1, 2, 9, 60, 200):
        # graded upper-triangular matrix, the shape of beta
        R = np.triu(rng.standard_normal((m, m))) * np.logspace(0, -8, m)[None, :]
        U = np.zeros((m, m), order="F")
        S = np.zeros(m)
        Rf = np.asfortranarray(R)
        assert shim.shim_svd(m, _p(Rf), _p(U), _p(S)) == 0
        ref = np.linalg.svd(R, compute_uv=False)
        assert np.all(np.diff(S) <= 0)
        assert np.abs(S - ref).max() <= 100 * m * EPS * ref[0]
        assert np.linalg.norm(U.T @ U - np.eye(m), 2) <= 1e-10
        # column i of U^T R has norm sigma_i
        assert np.allclose(np.linalg.norm(U.T @ R, axis=1), S, rtol=1e-8, atol=1e-12 * ref[0])


def test_solve_complex(shim):
    rng = np.random.default_rng(9)
    m = 37
    M = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    b = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    Mre, Mim = np.asfortranarray(M.real), np.asfortranarray(M.imag)
    bre, bim = b.real.copy(), b.imag.copy()
    assert shim.shim_solve(m, _p(Mre), _p(Mim), _p(bre), _p(bim)) == 0
    x = bre + 1j * bim
    assert np.abs(x - np.linalg.solve(M, b)).max() <= 1e-10
