"""Continuous Sylvester equation test problems (Section 4.3) and seeded right-hand sides.

Input generation only: the matrices of the section, random positive-real
tridiagonal matrices, manufactured solutions and C = A X* + X* B.  Tridiagonal
matrices are triples (sub[n-1], diag[n], sup[n-1]) with T[i+1, i] = sub[i] and
T[i, i+1] = sup[i].
"""
from __future__ import annotations

import numpy as np


def paper_tridiag(n: int, r: float):
    """A = B = M + 2 r N + 100/(n+1)^2 I with M = Tridiag(-1, 2, -1) and
    N = Tridiag(0.5, 0, -0.5) (Tridiag's arguments: sub, diagonal, super)."""
    return (np.full(n - 1, -1.0 + r), np.full(n, 2.0 + 100.0 / (n + 1) ** 2), np.full(n - 1, -1.0 - r))


def random_tridiag(n: int, seed: int, skew: float = 0.4):
    """Positive-real tridiagonal matrix: symmetric part strictly diagonally
    dominant, seeded random skew part (numpy PCG64)."""
    rng = np.random.default_rng(seed)
    off = rng.uniform(-1.0, -0.2, max(n - 1, 0))
    k = rng.uniform(-skew, skew, max(n - 1, 0))
    diag = 2.2 + rng.uniform(0.0, 0.5, n)
    return (off + k, diag, off - k)


def tridiag_apply_left(T, X):
    """T X (manufactures right-hand sides)."""
    sub, diag, sup = T
    Y = diag[:, None] * X
    Y[1:] += sub[:, None] * X[:-1]
    Y[:-1] += sup[:, None] * X[1:]
    return Y


def tridiag_apply_right(X, T):
    """X T (manufactures right-hand sides)."""
    sub, diag, sup = T
    Y = X * diag[None, :]
    Y[:, 1:] += X[:, :-1] * sup[None, :]
    Y[:, :-1] += X[:, 1:] * sub[None, :]
    return Y


def sylvester_rhs(A, B, kind: str = "ones", seed: int | None = None):
    """Manufactured X* (all ones, or U(-1, 1) seeded) and C = A X* + X* B."""
    m, n = len(A[1]), len(B[1])
    if kind == "ones":
        Xs = np.ones((m, n))
    elif kind == "uniform":
        Xs = np.random.default_rng(seed).uniform(-1.0, 1.0, (m, n))
    else:
        raise ValueError(kind)
    return Xs, tridiag_apply_left(A, Xs) + tridiag_apply_right(Xs, B)
