"""GADI-AB for the continuous Sylvester equation in float64 -- TEST INFRASTRUCTURE ONLY.

Section 4.3 applies GADI-IR to A X + X B = C (its residual is R = C - A X - X B)
with the splitting of L(X) = A X + X B into M(X) = A X and N(X) = X B ("M, N
replaced by A, B").  One sweep of Algorithm 1 in this setting:

    R = C - A X - X B                   (step 1, the residual)
    (alpha I + A) Z = R                 (step 2: one solve per column of R)
    Y (alpha I + B) = (2 - omega) alpha Z   (step 3: one solve per row)
    X <- X + Y                          (step 4)

Tridiagonal matrices are triples (sub[n-1], diag[n], sup[n-1]) with
T[i+1, i] = sub[i] and T[i, i+1] = sup[i].  The inner solves are scipy's banded
LU (LAPACK gbsv), exact up to rounding.  Nothing here is shared with the GPU
path.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def paper_matrix(n: int, r: float):
    """A = B = M + 2 r N + 100/(n+1)^2 I with M = Tridiag(-1, 2, -1) and
    N = Tridiag(0.5, 0, -0.5), Tridiag's arguments in (sub, diagonal, super)
    order: sub = -1 + r, diagonal = 2 + 100/(n+1)^2, super = -1 - r."""
    return (np.full(n - 1, -1.0 + r), np.full(n, 2.0 + 100.0 / (n + 1) ** 2), np.full(n - 1, -1.0 - r))


def dense(T) -> np.ndarray:
    sub, diag, sup = T
    return np.diag(diag) + np.diag(sub, -1) + np.diag(sup, 1)


def left(T, X):
    """T X for a tridiagonal T (rows of X are indexed by T)."""
    sub, diag, sup = T
    Y = diag[:, None] * X
    Y[1:] += sub[:, None] * X[:-1]
    Y[:-1] += sup[:, None] * X[1:]
    return Y


def right(X, T):
    """X T for a tridiagonal T (columns of X are indexed by T)."""
    sub, diag, sup = T
    Y = X * diag[None, :]
    # (X T)[:, j] = X[:, j-1] T[j-1, j] + X[:, j] T[j, j] + X[:, j+1] T[j+1, j]
    Y[:, 1:] += X[:, :-1] * sup[None, :]
    Y[:, :-1] += X[:, 1:] * sub[None, :]
    return Y


def _banded(T, alpha, transpose=False):
    sub, diag, sup = T
    if transpose:
        sub, sup = sup, sub
    n = len(diag)
    ab = np.zeros((3, n))
    ab[0, 1:] = sup
    ab[1, :] = diag + alpha
    ab[2, :-1] = sub
    return ab


def solve_left(T, alpha, R):
    """Z with (alpha I + T) Z = R."""
    return sla.solve_banded((1, 1), _banded(T, alpha), R)


def solve_right(T, alpha, G):
    """Y with Y (alpha I + T) = G, i.e. (alpha I + T)^T Y^T = G^T."""
    return sla.solve_banded((1, 1), _banded(T, alpha, transpose=True), G.T).T


def residual(A, B, C, X):
    """R = C - A X - X B (Section 4.3)."""
    return C - left(A, X) - right(X, B)


def gadi_ab(A, B, C, alpha, omega, tol=1e-10, maxit=20000, x0=None, plant=0):
    """GADI-AB from X_0 (zero by default) until ||R_k||_F <= tol ||R_0||_F.

    Returns dict(x, status in {'ok', 'maxit', 'diverged'}, sweeps, hist) with
    hist[k] = ||R_k||_F / ||R_0||_F.  plant = 1 solves step 3 from the wrong
    side ((alpha I + B) Y = G), a mistake the pins must catch."""
    X = np.zeros_like(C, dtype=np.float64) if x0 is None else np.array(x0, dtype=np.float64)
    hist = []
    rho0 = None
    status = "maxit"
    k = 0
    while True:
        R = residual(A, B, C, X)
        rho = np.linalg.norm(R)
        if rho0 is None:
            rho0 = rho
        hist.append(rho / rho0 if rho0 > 0 else 0.0)
        if rho <= tol * rho0:
            status = "ok"
            break
        if not np.isfinite(rho) or rho > 1e6 * rho0:
            status = "diverged"
            break
        if k >= maxit:
            break
        Z = solve_left(A, alpha, R)
        G = (2.0 - omega) * alpha * Z
        Y = solve_left(B, alpha, G) if plant == 1 else solve_right(B, alpha, G)
        X = X + Y
        k += 1
    return {"x": X, "status": status, "sweeps": k, "hist": np.array(hist)}


def kron_operators(A, B):
    """vec-form operators (column-major vec): L = I (x) A + B^T (x) I, M = I (x) A, N = B^T (x) I."""
    Ad, Bd = dense(A), dense(B)
    m, n = Ad.shape[0], Bd.shape[0]
    M = np.kron(np.eye(n), Ad)
    N = np.kron(Bd.T, np.eye(m))
    return M + N, M, N
