"""Host-side small eigensolvers of the library (complex Jacobi, generalised
Hermitian-definite problem, tridiagonal resolvent) against numpy, built with g++."""
import os
import subprocess
import tempfile

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def exe():
    d = tempfile.mkdtemp()
    out = os.path.join(d, "small_eig")
    subprocess.check_call(["g++", "-O2", "-std=c++17", os.path.join(HERE, "host", "small_eig_driver.cpp"), "-o", out])
    return out


def _run(exe, txt):
    return subprocess.run([exe], input=txt, capture_output=True, text=True, check=True).stdout.split("\n")


def _mat(M):
    return " ".join("%.17g %.17g" % (z.real, z.imag) for z in M.ravel())


def _herm(n, seed):
    r = np.random.default_rng(seed)
    A = r.standard_normal((n, n)) + 1j * r.standard_normal((n, n))
    return (A + A.conj().T) / 2


@pytest.mark.parametrize("n", [1, 2, 5, 12, 48])
def test_jacobi_matches_eigh(exe, n):
    A = _herm(n, n)
    lines = _run(exe, "0 %d %s" % (n, _mat(A)))
    w = np.array([float(x) for x in lines[:n]])
    V = np.array([complex(*map(float, l.split())) for l in lines[n:n + n * n]]).reshape(n, n)
    assert np.abs(w - np.linalg.eigvalsh(A)).max() < 1e-12 * max(1, np.abs(w).max())
    assert np.abs(V.conj().T @ V - np.eye(n)).max() < 1e-12
    assert np.abs(A @ V - V * w).max() < 1e-11


def test_jacobi_degenerate(exe):
    # repeated eigenvalues and an already diagonal block
    Q = np.linalg.qr(np.random.default_rng(1).standard_normal((6, 6)) + 1j * np.random.default_rng(2).standard_normal((6, 6)))[0]
    A = Q @ np.diag([1.0, 1.0, 1.0, -2.0, 3.0, 3.0]) @ Q.conj().T
    lines = _run(exe, "0 6 %s" % _mat(A))
    w = np.array([float(x) for x in lines[:6]])
    assert np.allclose(w, [-2, 1, 1, 1, 3, 3], atol=1e-12)


def test_generalised(exe):
    n = 9
    A = _herm(n, 3)
    B = np.random.default_rng(4).standard_normal((n, n)) + 1j * np.random.default_rng(5).standard_normal((n, n))
    G = B @ B.conj().T + n * np.eye(n)
    lines = _run(exe, "1 %d %s %s" % (n, _mat(A), _mat(G)))
    w = np.array([float(x) for x in lines[:n]])
    X = np.array([complex(*map(float, l.split())) for l in lines[n:n + n * n]]).reshape(n, n)
    import scipy.linalg
    assert np.abs(w - scipy.linalg.eigh(A, G, eigvals_only=True)).max() < 1e-11
    assert np.abs(X.conj().T @ G @ X - np.eye(n)).max() < 1e-10
    assert np.abs(A @ X - G @ X * w).max() < 1e-10


def test_tridiagonal_resolvent(exe):
    m = 7
    r = np.random.default_rng(6)
    a, b = r.standard_normal(m), np.r_[0.0, r.random(m - 1) + 0.1]
    z = 0.3 + 0.1j
    lines = _run(exe, "2 %d %s %s 1.7 %.17g %.17g" % (m, " ".join("%.17g" % x for x in a), " ".join("%.17g" % x for x in b), z.real, z.imag))
    s = np.array([complex(*map(float, l.split())) for l in lines[:m]])
    T = np.diag(a) + np.diag(b[1:], 1) + np.diag(b[1:], -1)
    e1 = np.zeros(m)
    e1[0] = 1.7
    assert np.abs(s - np.linalg.solve(z * np.eye(m) - T, e1)).max() < 1e-12


def test_generalised_rank_deficient(exe):
    # Gram matrix of 6 vectors spanning only 4 dimensions: the rank-revealing
    # solver returns the 4 Ritz values of A restricted to that span
    n, r = 6, 4
    rng = np.random.default_rng(7)
    S = rng.standard_normal((10, r)) + 1j * rng.standard_normal((10, r))
    S = np.concatenate([S, S[:, :2] @ (rng.standard_normal((2, 2)) + 0j)], axis=1)   # 6 columns, rank 4
    H = _herm(10, 8)
    A, G = S.conj().T @ H @ S, S.conj().T @ S
    lines = _run(exe, "3 %d %s %s" % (n, _mat(A), _mat(G)))
    rank = int(lines[0])
    w = np.array([float(x) for x in lines[1:1 + rank]])
    Q = np.linalg.qr(S[:, :r])[0]
    ref = np.linalg.eigvalsh(Q.conj().T @ H @ Q)
    assert rank == r
    assert np.abs(w - ref).max() < 1e-9


@pytest.mark.parametrize("n,kind", [(1, "rand"), (2, "rand"), (7, "rand"), (40, "rand"), (64, "zero_diag"),
                                    (200, "zero_diag"), (30, "graded"), (12, "split")])
def test_tridiagonal_eigen_first_components(exe, n, kind):
    r = np.random.default_rng(n)
    d = r.standard_normal(n)
    e = r.random(max(n - 1, 0)) + 0.1
    if kind == "zero_diag":          # the structure of the full-BSE Lanczos tridiagonal: +-theta pairs
        d[:] = 0.0
    if kind == "graded":
        d = d * 10.0 ** np.linspace(0, 8, n)
        e = e * 10.0 ** np.linspace(0, 7, n - 1)
    if kind == "split":
        e[5] = 0.0
    lines = _run(exe, "4 %d %s %s" % (n, " ".join("%.17g" % x for x in d), " ".join("%.17g" % x for x in e)))
    w = np.array([float(x) for x in lines[:n]])
    z = np.array([float(x) for x in lines[n:2 * n]])
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    ref_w, ref_V = np.linalg.eigh(T)
    scale = max(1.0, np.abs(ref_w).max())
    assert np.abs(w - ref_w).max() < 1e-12 * scale
    if kind == "zero_diag":
        assert np.abs(w + w[::-1]).max() < 1e-12 * scale
    # first components: z_i^2 are the quadrature weights (sum 1); compare where eigenvalues are simple
    assert abs((z ** 2).sum() - 1.0) < 1e-12
    gap = np.diff(ref_w)
    simple = np.ones(n, bool)
    simple[:-1] &= gap > 1e-8 * scale
    simple[1:] &= gap > 1e-8 * scale
    assert np.abs(z[simple] ** 2 - ref_V[0, simple] ** 2).max() < 1e-10
