"""Pins of the GADI-AB oracle (Section 4.3, continuous Sylvester equation), CPU only.

S1  the fixed point is the solution of A X + X B = C (Bartels-Stewart, scipy) on a
    non-square system (a transposition mistake changes the answer);
S2  one sweep equals the GADI framework equation (Section 2.1) with M = I (x) A and
    N = B^T (x) I written out with dense Kronecker operators; a planted mistake
    (step 3 solved from the wrong side) fails it;
S3  symmetric case r = 0: the solution in the DST-I eigenbasis, X^ = C^ / (l_i + l_j),
    independent of any library Sylvester solver;
S4  the observed contraction rate matches the spectral radius of the iteration
    matrix I - (2 - omega) alpha (alpha I + N)^-1 (alpha I + M)^-1 L (within 5%);
S5  the paper's matrix M + 2 r N + 100/(n+1)^2 I built from its definition.
"""
import numpy as np
import pytest
import scipy.fft
import scipy.linalg as sla

from oracle import sylvester as syl


def rand_tridiag(n, seed, skew=0.4):
    """Positive-real tridiagonal: symmetric part diagonally dominant, random skew part."""
    rng = np.random.default_rng(seed)
    off = rng.uniform(-1.0, -0.2, n - 1)
    k = rng.uniform(-skew, skew, n - 1)
    diag = 2.2 + rng.uniform(0.0, 0.5, n)
    return (off + k, diag, off - k)


@pytest.mark.parametrize("alpha,omega", [(0.5, 0.5), (2.0, 0.0), (0.3, 1.2)])
def test_s1_fixed_point_is_the_sylvester_solution(alpha, omega):
    m, n = 11, 13
    A, B = rand_tridiag(m, 1), rand_tridiag(n, 2)
    C = np.random.default_rng(3).normal(size=(m, n))
    res = syl.gadi_ab(A, B, C, alpha, omega, tol=1e-13, maxit=5000)
    assert res["status"] == "ok"
    Xref = sla.solve_sylvester(syl.dense(A), syl.dense(B), C)
    assert np.linalg.norm(res["x"] - Xref) <= 1e-10 * np.linalg.norm(Xref)


def _framework_sweep(L, M, N, b, x, alpha, omega):
    I = np.eye(len(b))
    xh = np.linalg.solve(alpha * I + M, (alpha * I - N) @ x + b)
    return np.linalg.solve(alpha * I + N, (N - (1.0 - omega) * alpha * I) @ x + (2.0 - omega) * alpha * xh)


@pytest.mark.parametrize("m,n,plant", [(5, 7, 0), (6, 6, 0), (6, 6, 1)])
def test_s2_one_sweep_is_the_framework_equation(m, n, plant):
    A, B = rand_tridiag(m, 4), rand_tridiag(n, 5)
    C = np.random.default_rng(6).normal(size=(m, n))
    L, M, N = syl.kron_operators(A, B)
    X0 = np.random.default_rng(7).normal(size=(m, n))
    alpha, omega = 0.7, 0.4
    res = syl.gadi_ab(A, B, C, alpha, omega, tol=0.0, maxit=1, x0=X0, plant=plant)
    x1 = _framework_sweep(L, M, N, C.flatten(order="F"), X0.flatten(order="F"), alpha, omega)
    err = np.linalg.norm(res["x"].flatten(order="F") - x1) / np.linalg.norm(x1)
    if plant == 0:
        assert err <= 1e-12
    else:
        assert err > 1e-3


def test_s3_symmetric_case_in_the_sine_basis():
    n = 20
    A = syl.paper_matrix(n, 0.0)
    C = np.random.default_rng(8).normal(size=(n, n))
    res = syl.gadi_ab(A, A, C, 0.5, 0.5, tol=1e-14, maxit=5000)
    assert res["status"] == "ok"
    # A = Tridiag(-1, d, -1): eigenvalues d - 2 cos(j pi/(n+1)), orthonormal DST-I eigenvectors
    d = A[1][0]
    lam = d - 2.0 * np.cos(np.arange(1, n + 1) * np.pi / (n + 1))
    Ch = scipy.fft.dstn(C, type=1, norm="ortho")
    X = scipy.fft.idstn(Ch / (lam[:, None] + lam[None, :]), type=1, norm="ortho")
    assert np.linalg.norm(res["x"] - X) <= 1e-11 * np.linalg.norm(X)


def test_s4_rate_is_the_spectral_radius():
    n = 8
    A = syl.paper_matrix(n, 0.5)
    C = np.random.default_rng(9).normal(size=(n, n))
    alpha, omega = 0.4, 0.5
    L, M, N = syl.kron_operators(A, A)
    I = np.eye(n * n)
    T = I - (2.0 - omega) * alpha * np.linalg.solve(alpha * I + N, np.linalg.solve(alpha * I + M, L))
    rho = max(abs(np.linalg.eigvals(T)))
    assert rho < 1.0
    res = syl.gadi_ab(A, A, C, alpha, omega, tol=1e-13, maxit=20000)
    h = res["hist"]
    k = len(h) - 1
    rate = (h[k] / h[k // 2]) ** (1.0 / (k - k // 2))
    assert abs(rate - rho) <= 0.05 * rho, (rate, rho)


def test_s5_paper_matrix():
    n, r = 6, 0.3
    M = 2 * np.eye(n) - np.eye(n, k=-1) - np.eye(n, k=1)
    N = 0.5 * np.eye(n, k=-1) - 0.5 * np.eye(n, k=1)
    ref = M + 2 * r * N + 100.0 / (n + 1) ** 2 * np.eye(n)
    assert np.array_equal(syl.dense(syl.paper_matrix(n, r)), ref)


def test_products_match_dense():
    A, B = rand_tridiag(6, 10), rand_tridiag(4, 11)
    X = np.random.default_rng(12).normal(size=(6, 4))
    assert np.allclose(syl.left(A, X), syl.dense(A) @ X, rtol=1e-14, atol=1e-14)
    assert np.allclose(syl.right(X, B), X @ syl.dense(B), rtol=1e-14, atol=1e-14)
