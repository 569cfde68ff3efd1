"""Parity at the benchmark sizes, in the launch configuration bench.py times.

The 3-D 128^3 (beta = 20, x* ~ U(-1, 1) seed 0) and 256^3 (beta ~ U(0, 100) per
axis, x* = 1) systems are too large for a full oracle solve in a test, so the
checks are (i) sampled rows of every packed operator against the oracle's row
computed one by one from the CSR of A, and (ii) properties that hold at any
size: the FP64 residual of the GPU solution, recomputed by the oracle's SpMV on
the CPU, is <= tol, and the relative error against the manufactured solution
obeys the forward-error bound ||x - x*|| <= ||r|| / lambda_min(H) (A is
positive real, so sigma_min(A) >= lambda_min(H), which has a closed form).
"""
import math

import numpy as np
import pytest

import gadi_inputs as gi
import oracle
from oracle import dense as od

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2501_04229_amd as gadi  # noqa: E402

U16 = 2.0 ** -11
U32 = 2.0 ** -24


@pytest.fixture(scope="module", params=["convdiff3d_128_beta20", "convdiff3d_256_betaU100"])
def big(request):
    W = gi.workload(request.param)
    A = W["A"]
    g = gadi.System(A)
    yield request.param, W, g
    g.close()


def _rows_sample(n, k, seed):
    rng = np.random.default_rng(seed)
    edge = np.array([0, 1, n - 2, n - 1])
    return np.unique(np.concatenate([edge, rng.integers(0, n, size=k)]))


def test_sampled_rows_of_products(big):
    """Each packed operator row equals the row computed from A's CSR (H, S formed from A and A^T)."""
    name, W, g = big
    A = W["A"]
    n = A.n
    rows = _rows_sample(n, 3000, 5)
    rng = np.random.default_rng(9)
    x16 = rng.uniform(-1, 1, n).astype(np.float16)
    x64 = rng.uniform(-1, 1, n)
    xd16 = torch.from_numpy(x16.view(np.int16)).cuda().view(torch.float16)
    xd64 = torch.from_numpy(x64).cuda()
    yA = torch.empty_like(xd64)
    yH = torch.empty_like(xd16)
    yS = torch.empty_like(xd16)
    alpha = 0.5
    g.spmv("A", xd64, yA)
    g.spmv("H16", xd16, yH, alpha)
    g.spmv("S16", xd16, yS, alpha)
    torch.cuda.synchronize()
    yA = yA.cpu().numpy()
    yH = yH.cpu().numpy().astype(np.float64)
    yS = yS.cpu().numpy().astype(np.float64)
    rp, col, val = A.row_ptr, A.col, A.val
    xv = x16.astype(np.float64)
    for i in rows:
        cols = col[rp[i]:rp[i + 1]]
        a_row = val[rp[i]:rp[i + 1]]
        # A x in double
        ref = float(np.dot(a_row, x64[cols]))
        assert abs(yA[i] - ref) <= 8 * 2.0 ** -53 * float(np.dot(np.abs(a_row), np.abs(x64[cols]))) + 1e-300
        # row i of H and S from A_ij and A_ji (A_ji read from row j)
        h = {}
        s = {}
        for j, aij in zip(cols, a_row):
            cj = col[rp[j]:rp[j + 1]]
            k = np.searchsorted(cj, i)
            aji = val[rp[j] + k] if k < len(cj) and cj[k] == i else 0.0
            h[j] = np.float16((aij + aji) / 2.0)
            s[j] = np.float16((aij - aji) / 2.0)
        hr = alpha * xv[i] + sum(float(h[j]) * xv[j] for j in h)
        hm = alpha * abs(xv[i]) + sum(abs(float(h[j]) * xv[j]) for j in h)
        assert abs(yH[i] - hr) <= (U16 + 10 * U32) * hm + 6e-8, (name, i)
        sr = xv[i] + sum(float(s[j]) * xv[j] for j in s if j != i) / alpha
        sm = abs(xv[i]) + sum(abs(float(s[j]) * xv[j]) for j in s if j != i) / alpha
        assert abs(yS[i] - sr) <= (U16 + 10 * U32) * sm + 6e-8, (name, i)


@pytest.mark.parametrize("prec", ["fp16", "fp8"])
def test_fullsize_fp16_solve_properties(big, prec):
    """FP16-IR (and the FP8 storage mode) from x = 0 to RES <= 1e-10 at (0.5, 0.5) on the device-resident
    right-hand side."""
    name, W, g = big
    A, b, xs = W["A"], W["b"], W["xstar"]
    bd = torch.from_numpy(b).cuda()
    x, info = g.solve(bd, 0.5, 0.5, tol=1e-10, prec=prec)
    torch.cuda.synchronize()
    assert info["status"] == gadi.OK, info
    xh = x.cpu().numpy()
    o = oracle.OracleSystem(A)
    r = b - o.spmv("A", xh)
    rel = np.linalg.norm(r) / np.linalg.norm(b)
    assert rel <= 1.0000001e-10, rel
    n = A.grid
    lmin = 3 * (2.0 - 2.0 * math.cos(math.pi / (n + 1)))
    err = np.linalg.norm(xh - xs)
    assert err <= np.linalg.norm(r) / lmin * 1.0000001, (err, np.linalg.norm(r) / lmin)
    assert err / np.linalg.norm(xs) <= 1e-6
