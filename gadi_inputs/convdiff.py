"""Convection-diffusion test matrices and seeded workloads.

The matrix family is the one of the paper's Section 4.1: centred differences of
-Laplace(u) + beta . grad(u) on the unit square/cube with homogeneous Dirichlet
boundary, written without the 1/h^2 factor, i.e.

    A = T_x (x) I (x) I + I (x) T_y (x) I + I (x) I (x) T_z        (3-D)
    A = T_x (x) I + I (x) T_y                                      (2-D)

with T_x = Tridiag(-1 - r_x, 2*dim, -1 + r_x) and T_y, T_z = Tridiag(-1 - r, 0,
-1 + r), where r_a = beta_a * h / 2 = beta_a / (2 (n + 1)).  The paper uses a
single beta = 1 (so r = 1/(2n+2)); the per-axis beta generalises it.

Unknowns are ordered lexicographically with x the slowest index (the
Kronecker order above): idx = (i_x * n + i_y) * n + i_z, 0-based.  Columns
within a row are sorted ascending.

Everything here is input generation; no solver arithmetic lives in this file.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Sequence

import numpy as np

# (alpha, omega) trial grid of the batched parameter sweep: 4 log-spaced alphas
# over [1e-3, 10] times 4 omegas.
ALPHA_GRID = tuple(float(a) for a in np.logspace(-3.0, 1.0, 4))
OMEGA_GRID = (0.0, 0.5, 1.0, 1.5)


@dataclasses.dataclass
class Csr:
    """Square CSR matrix with int32 indices and float64 values."""

    n: int
    row_ptr: np.ndarray  # int32 [n+1]
    col: np.ndarray      # int32 [nnz]
    val: np.ndarray      # float64 [nnz]
    dim: int = 0
    grid: int = 0
    beta: tuple = ()

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))


def _beta_tuple(beta, dim: int) -> tuple:
    if np.ndim(beta) == 0:
        return tuple(float(beta) for _ in range(dim))
    b = tuple(float(v) for v in beta)
    if len(b) != dim:
        raise ValueError(f"beta needs {dim} entries, got {len(b)}")
    return b


def convdiff_nnz(n: int, dim: int) -> int:
    """Closed-form nnz: (2 dim + 1) n^dim - 2 dim n^(dim-1)."""
    return (2 * dim + 1) * n ** dim - 2 * dim * n ** (dim - 1)


def convdiff(n: int, dim: int, beta) -> Csr:
    """Build the h^2-scaled convection-diffusion matrix on an n^dim interior grid."""
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    if n < 1:
        raise ValueError("n must be >= 1")
    beta_t = _beta_tuple(beta, dim)
    r = [b / (2.0 * (n + 1)) for b in beta_t]
    N = n ** dim
    strides = [n ** (dim - 1 - a) for a in range(dim)]
    idx = np.arange(N, dtype=np.int64)
    coord = [(idx // strides[a]) % n for a in range(dim)]

    # stencil slots in ascending column order: lower neighbours from the
    # slowest axis to the fastest, the diagonal, upper neighbours back out.
    slots = []  # (offset, coefficient, validity mask or None)
    for a in range(dim):
        slots.append((-strides[a], -1.0 - r[a], coord[a] >= 1))
    slots.append((0, float(2 * dim), None))
    for a in reversed(range(dim)):
        slots.append((strides[a], -1.0 + r[a], coord[a] <= n - 2))

    k = len(slots)
    mask = np.ones((N, k), dtype=bool)
    cols = np.empty((N, k), dtype=np.int32)
    vals = np.empty((N, k), dtype=np.float64)
    for j, (off, coef, valid) in enumerate(slots):
        cols[:, j] = (idx + off).astype(np.int32) if off else idx.astype(np.int32)
        vals[:, j] = coef
        if valid is not None:
            mask[:, j] = valid
    del coord
    counts = mask.sum(axis=1, dtype=np.int64)
    row_ptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col = cols[mask]
    val = vals[mask]
    del cols, vals, mask
    if row_ptr[-1] >= 2 ** 31:
        raise ValueError("nnz does not fit int32")
    return Csr(N, row_ptr.astype(np.int32), col, val, dim=dim, grid=n, beta=beta_t)


def convdiff_skew_perturbed(n: int, dim: int, beta, extra_per_row: float, scale: float, seed: int,
                            rows_fraction: float = 1.0) -> Csr:
    """Convection-diffusion matrix plus a random skew-symmetric perturbation
    scale * (R - R^T), R with about `extra_per_row` random off-diagonal entries
    in a `rows_fraction` of the rows.  H = (A + A^T)/2 is unchanged (still SPD),
    the pattern is irregular: an input for the explicit-column storage path."""
    import scipy.sparse as sp
    A = convdiff(n, dim, beta).to_scipy().tocoo()
    N = A.shape[0]
    rng = np.random.default_rng(seed)
    rows = np.flatnonzero(rng.random(N) < rows_fraction)
    k = int(round(extra_per_row * len(rows)))
    ri = rng.choice(rows, size=k) if len(rows) else np.zeros(0, dtype=np.int64)
    ci = rng.integers(0, N, size=k)
    keep = ri != ci
    ri, ci = ri[keep], ci[keep]
    v = rng.uniform(-1.0, 1.0, size=len(ri))
    R = sp.coo_matrix((v, (ri, ci)), shape=(N, N)).tocsr()
    M = (A.tocsr() + scale * (R - R.T)).tocsr()
    M.sum_duplicates()
    M.sort_indices()
    return Csr(N, M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(np.float64),
               dim=dim, grid=n, beta=_beta_tuple(beta, dim))


def csr_matvec(A: Csr, x: np.ndarray) -> np.ndarray:
    """y = A x in float64 (used only to manufacture right-hand sides)."""
    return A.to_scipy() @ np.asarray(x, dtype=np.float64)


def rhs_for(A: Csr, kind: str = "ones", seed: int | None = None):
    """Manufactured solution x* and b = A x*.

    kind = "ones": x* = (1, ..., 1) as in the paper; kind = "uniform":
    x* ~ U(-1, 1) from numpy's PCG64 generator seeded with `seed`.
    """
    if kind == "ones":
        xs = np.ones(A.n)
    elif kind == "uniform":
        xs = np.random.default_rng(seed).uniform(-1.0, 1.0, A.n)
    else:
        raise ValueError(kind)
    return xs, csr_matvec(A, xs)


def workload(name: str) -> dict:
    """Named single-system workloads.

    convdiff2d_64_beta10     : 2-D, n = 64, beta = 10, b = A 1, (alpha, omega) = (0.5, 0.5)
    convdiff3d_128_beta20    : 3-D, n = 128, beta = (20, 20, 20), x* ~ U(-1,1) seed 0
    convdiff3d_256_betaU100  : 3-D, n = 256, beta ~ U(0, 100) per axis (seed 1), x* = 1
    convdiff3d_<n>_beta<b>   : any other size, x* = 1
    """
    if name == "convdiff2d_64_beta10":
        A = convdiff(64, 2, 10.0)
        xs, b = rhs_for(A, "ones")
    elif name == "convdiff3d_128_beta20":
        A = convdiff(128, 3, 20.0)
        xs, b = rhs_for(A, "uniform", 0)
    elif name == "convdiff3d_256_betaU100":
        beta = np.random.default_rng(1).uniform(0.0, 100.0, 3)
        A = convdiff(256, 3, beta)
        xs, b = rhs_for(A, "ones")
    elif name.startswith("convdiff3d_") or name.startswith("convdiff2d_"):
        dim = 3 if name.startswith("convdiff3d_") else 2
        parts = name.split("_")
        n = int(parts[1])
        beta = float(parts[2].replace("beta", ""))
        A = convdiff(n, dim, beta)
        xs, b = rhs_for(A, "ones")
    else:
        raise KeyError(name)
    return {"name": name, "A": A, "b": b, "xstar": xs, "alpha": 0.5, "omega": 0.5}


def batched_family(count: int = 64, seed: int = 2, nmin: int = 128, nmax: int = 1024):
    """Uneven 2-D systems for the batched sweep: n ~ U{nmin..nmax}, beta ~ logU(1, 1000).

    Returns a list of (n, dim, beta).  One generator draws n then beta per
    system, in that order.
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.integers(nmin, nmax + 1))
        beta = float(10.0 ** rng.uniform(0.0, 3.0))
        out.append((n, 2, beta))
    return out


def train_family(count: int = 256, seeds: Sequence[int] = (10, 11, 12, 13)):
    """Small training systems for the (alpha, omega) predictor.

    Three in four are 3-D (n ~ U{16..96}), one in four 2-D (n ~ U{32..160});
    beta ~ logU(1, 500) drawn per axis.  Systems of the same structure as the
    large ones but up to 1800 times smaller, as the paper's training-set
    generation prescribes.  One generator per seed draws n, then beta.
    """
    out = []
    per = count // len(seeds)
    for s in seeds:
        rng = np.random.default_rng(s)
        for i in range(per):
            dim = 2 if (i % 4 == 0) else 3
            n = int(rng.integers(32, 161)) if dim == 2 else int(rng.integers(16, 97))
            beta = tuple(float(10.0 ** rng.uniform(0.0, math.log10(500.0))) for _ in range(dim))
            out.append((n, dim, beta))
    return out


def test_family(count: int = 40, seed: int = 4, nmin: int = 96, nmax: int = 192):
    """Fresh 3-D systems for the predictor's evaluation: n ~ U{nmin..nmax}, beta ~ logU(1, 500)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(nmin, nmax + 1))
        beta = float(10.0 ** rng.uniform(0.0, math.log10(500.0)))
        out.append((n, 3, beta, seed + i))
    return out
