"""Dense float64 forms of GADI for tiny grids -- TEST INFRASTRUCTURE ONLY.

Used to pin the C oracle.  Each function writes one formula of the paper out
with numpy's dense solver; nothing here is shared with the GPU path.
"""
from __future__ import annotations

import numpy as np


def dense(A) -> np.ndarray:
    """CSR (gadi_inputs.Csr) -> dense float64 array."""
    M = np.zeros((A.n, A.n))
    for i in range(A.n):
        for k in range(A.row_ptr[i], A.row_ptr[i + 1]):
            M[i, A.col[k]] += A.val[k]
    return M


def hss(Ad: np.ndarray):
    """H = (A + A^T)/2, S = (A - A^T)/2 (the Section 4.1 splitting)."""
    return (Ad + Ad.T) / 2.0, (Ad - Ad.T) / 2.0


def gadi_stationary(Ad, b, alpha, omega, sweeps, x0=None):
    """The GADI framework equation of Section 2.1 with M = H, N = S:
        (alpha I + M) x_half = (alpha I - N) x_k + b
        (alpha I + N) x_{k+1} = (N - (1 - omega) alpha I) x_k + (2 - omega) alpha x_half
    Returns the list of iterates x_0 .. x_sweeps."""
    M, N = hss(Ad)
    n = Ad.shape[0]
    I = np.eye(n)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=float)
    out = [x.copy()]
    for _ in range(sweeps):
        xh = np.linalg.solve(alpha * I + M, (alpha * I - N) @ x + b)
        x = np.linalg.solve(alpha * I + N, (N - (1.0 - omega) * alpha * I) @ x + (2.0 - omega) * alpha * xh)
        out.append(x.copy())
    return out


def gadi_correction(Ad, b, alpha, omega, sweeps=None, tol=None, x0=None, maxit=100000):
    """Algorithm 1 of Section 2.1 with exact inner solves, all in double:
        r = b - A x;  H z = r;  S y = (2 - omega) alpha z;  x = x + y
    with H, S the shifted operators alpha I + M, alpha I + N.
    Runs `sweeps` corrections, or until ||r|| <= tol ||r_0||.
    Returns (iterates, residual-history)."""
    M, N = hss(Ad)
    n = Ad.shape[0]
    I = np.eye(n)
    Hs, Ss = alpha * I + M, alpha * I + N
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=float)
    its, res = [x.copy()], []
    r0 = None
    k = 0
    while True:
        r = b - Ad @ x
        rn = np.linalg.norm(r)
        if r0 is None:
            r0 = rn
        res.append(rn / r0 if r0 > 0 else 0.0)
        if sweeps is not None and k >= sweeps:
            break
        if tol is not None and rn <= tol * r0:
            break
        if k >= maxit:
            break
        z = np.linalg.solve(Hs, r)
        y = np.linalg.solve(Ss, (2.0 - omega) * alpha * z)
        x = x + y
        its.append(x.copy())
        k += 1
    return its, np.array(res)


def iteration_matrix(Ad, alpha, omega):
    """Theorem 1: T = (alpha I + N)^-1 (alpha I + M)^-1 (alpha^2 I + M N - (1 - omega) alpha A)."""
    M, N = hss(Ad)
    n = Ad.shape[0]
    I = np.eye(n)
    rhs = alpha * alpha * I + M @ N - (1.0 - omega) * alpha * Ad
    return np.linalg.solve(alpha * I + N, np.linalg.solve(alpha * I + M, rhs))


def iteration_matrix_correction(Ad, alpha, omega):
    """Error propagator of the correction form: I - (2 - omega) alpha (alpha I + N)^-1 (alpha I + M)^-1 A."""
    M, N = hss(Ad)
    n = Ad.shape[0]
    I = np.eye(n)
    return I - (2.0 - omega) * alpha * np.linalg.solve(alpha * I + N, np.linalg.solve(alpha * I + M, Ad))


def spectral_radius(T) -> float:
    return float(np.max(np.abs(np.linalg.eigvals(T))))


def convdiff_eigs_H(n, dim):
    """Closed-form eigenvalues of H for the convection-diffusion family:
    sum over axes of (2 - 2 cos(j_a pi h)), j_a = 1..n, h = 1/(n+1)."""
    h = 1.0 / (n + 1)
    one = 2.0 - 2.0 * np.cos(np.arange(1, n + 1) * np.pi * h)
    grids = np.meshgrid(*([one] * dim), indexing="ij")
    return np.sort(sum(grids).ravel())


def convdiff_eigs_S_imag(n, dim, beta):
    """Closed-form eigenvalues of S (purely imaginary): i * sum_a 2 r_a cos(j_a pi h)."""
    h = 1.0 / (n + 1)
    beta = np.broadcast_to(np.asarray(beta, dtype=float), (dim,))
    parts = [2.0 * (beta[a] * h / 2.0) * np.cos(np.arange(1, n + 1) * np.pi * h) for a in range(dim)]
    grids = np.meshgrid(*parts, indexing="ij")
    return np.sort(sum(grids).ravel())


def hss_contraction_bound(n, dim, alpha):
    """Bai-Golub-Ng bound for HSS (omega = 0): max over eig(H) of |alpha - l| / (alpha + l)."""
    lam = convdiff_eigs_H(n, dim)
    return float(np.max(np.abs(alpha - lam) / (alpha + lam)))


def dst1_modes(n, dim):
    """Orthonormal DST-I basis matrix for one axis (columns are eigenvectors of Tridiag(-1, c, -1))."""
    j = np.arange(1, n + 1)
    return np.sqrt(2.0 / (n + 1)) * np.sin(np.outer(j, j) * np.pi / (n + 1))
