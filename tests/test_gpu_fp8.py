"""GPU parity of the FP8 storage mode (GADI_PREC_FP8_IR: E4M3 off-diagonal
values of H and S, half diagonal and vectors) against the CPU oracle.

- the E4M3 codes the library encodes equal the oracle's rounding of the
  oracle's H and S bit for bit (off-diagonal entries, CSR order);
- the FP8 product (alpha I + H) x, row by row, against the float64 product of
  the same decoded values within one half rounding plus fp32 accumulation;
- FP8-IR solves reach the FP64 residual tolerance (recomputed by the oracle)
  and the oracle's solution to relative 1e-8;
- entries beyond the E4M3 range give EOVERFLOW16 while FP16-IR still solves.
"""
import numpy as np
import pytest

import gadi_inputs as gi
import oracle
from oracle import fp8 as ofp8

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2501_04229_amd as gadi  # noqa: E402

U16 = 2.0 ** -11
U32 = 2.0 ** -24


def banded(n, offsets, seed):
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    A = sp.diags([np.full(n, 2.0 + 2 * len(offsets))], [0], shape=(n, n), format="lil")
    for d in offsets:
        k = rng.uniform(-0.5, 0.5, n - d)
        A.setdiag(-1.0 + k, d)
        A.setdiag(-1.0 - k, -d)
    A = A.tocsr()
    A.sort_indices()
    return gi.Csr(n, A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float64))


CASES = [
    ("2d64_b10", lambda: gi.convdiff(64, 2, 10.0)),
    ("3d17_b", lambda: gi.convdiff(17, 3, (3.0, 40.0, 0.5))),  # subnormal E4M3 values on one axis
    ("2d40_rand", lambda: gi.convdiff_skew_perturbed(40, 2, 5.0, 3.0, 0.2, seed=3)),
    ("band8", lambda: banded(3001, (1, 2, 37, 300), seed=5)),
]


@pytest.fixture(scope="module", params=CASES, ids=[c[0] for c in CASES])
def case(request):
    A = request.param[1]()
    return A, gadi.System(A), oracle.OracleSystem(A)


def _offdiag(rp, col, val):
    keep = np.ones(len(col), bool)
    for i in range(len(rp) - 1):
        keep[rp[i]:rp[i + 1]] &= col[rp[i]:rp[i + 1]] != i
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    return rows[keep], col[keep], val[keep]


def test_codes_match_the_oracle_rounding(case):
    A, g, o = case
    for which in ("H", "S"):
        rp, col, codes = g.split_fp8(which)
        orp, ocol, oval = o.split(which)
        r0, c0, v0 = _offdiag(orp, ocol, oval)
        ref, over = ofp8.round_e4m3(v0)
        assert not over.any()
        dev = {(int(i), int(c)): int(v) for i, c, v in zip(np.repeat(np.arange(A.n), np.diff(rp)), col, codes)}
        got = np.array([dev.get((int(i), int(c)), 0) for i, c in zip(r0, c0)], dtype=np.uint8)
        assert np.array_equal(got, ref), which
        # anything else the device stores is zero
        assert sum(1 for v in dev.values() if v & 0x7F) <= int(np.count_nonzero(ref & 0x7F))


@pytest.mark.parametrize("alpha", [1e-3, 0.5, 10.0])
def test_fp8_product(case, alpha):
    A, g, o = case
    rng = np.random.default_rng(14)
    x16 = rng.uniform(-1, 1, A.n).astype(np.float16)
    xd = torch.from_numpy(x16.view(np.int16)).cuda().view(torch.float16)
    yd = torch.empty_like(xd)
    g.spmv("H8", xd, yd, alpha)
    torch.cuda.synchronize()
    y = yd.cpu().numpy().astype(np.float64)
    orp, ocol, oval = o.split("H")
    q = oval.copy()
    rows = np.repeat(np.arange(A.n), np.diff(orp))
    off = ocol != rows
    q[off] = ofp8.decode(ofp8.round_e4m3(oval[off])[0])
    q[~off] = oval[~off].astype(np.float16).astype(np.float64)
    import scipy.sparse as sp
    M = sp.csr_matrix((q, ocol, orp), shape=(A.n, A.n))
    xv = x16.astype(np.float64)
    yref = alpha * xv + M @ xv
    mag = alpha * np.abs(xv) + abs(M) @ np.abs(xv)
    assert np.all(np.abs(y - yref) <= (U16 + 8 * U32) * mag + 6e-8)


def _lambda_min_h(A):
    from oracle import dense as od
    if A.grid:
        return od.convdiff_eigs_H(A.grid, A.dim)[0]
    lmin = oracle.OracleSystem(A).gershgorin()[0]
    assert lmin > 0
    return lmin


def test_fp8_solve_parity(case):
    A, g, o = case
    xs, b = gi.rhs_for(A, "uniform", 0)
    r = o.gadi(b, 0.5, 0.5, tol=1e-13, eps_h=1e-10, eps_s=1e-10)
    assert r["status"] == "ok"
    xref = r["x"]
    tol = min(1e-10, 0.9 * (1e-8 * _lambda_min_h(A) * np.linalg.norm(xref) / np.linalg.norm(b) - 1e-13))
    assert tol >= 1e-12
    x, info = g.solve(b, 0.5, 0.5, tol=tol, prec="fp8")
    assert info["status"] == gadi.OK, info
    rel = np.linalg.norm(b - o.spmv("A", x)) / np.linalg.norm(b)
    assert rel <= tol * 1.0000001, (rel, info)
    err = np.linalg.norm(x - xref) / np.linalg.norm(xref)
    assert err <= 1e-8, (err, tol, info)


def test_fp8_overflow_is_reported():
    A = gi.convdiff(8, 2, 1.0)
    big = gi.Csr(A.n, A.row_ptr, A.col, A.val * 500.0)  # off-diagonals near -500: beyond 448
    g = gadi.System(big)
    xs, b = gi.rhs_for(big, "ones")
    x, info = g.solve(b, 0.5 * 500.0, 0.5, tol=1e-10, prec="fp8")
    assert info["status"] == gadi.EOVERFLOW16, info
    x, info = g.solve(b, 0.5 * 500.0, 0.5, tol=1e-10, prec="fp16")
    assert info["status"] == gadi.OK, info
    with pytest.raises(gadi.GadiError):
        g.split_fp8("H")
