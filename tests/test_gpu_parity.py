"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Kernel-level products are checked row by row against float64 products of the
same rounded inputs with the bound of the arithmetic; solves are checked
against the oracle's solution (relative 1e-8) and must reach FP64 relative
residual 1e-10, recomputed on the CPU by the oracle.
"""
import math

import numpy as np
import pytest

import gadi_inputs as gi
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2501_04229_amd as gadi  # noqa: E402

U16 = 2.0 ** -11
U32 = 2.0 ** -24
U64 = 2.0 ** -53

def banded(n, offsets, seed):
    """Positive-real band matrix: diagonal 2 + 2 len(offsets), symmetric part -1 and
    a seeded skew part in (-0.5, 0.5) on each offset pair +-d."""
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
    ("3d17_b", lambda: gi.convdiff(17, 3, (3.0, 40.0, 0.5))),  # 4913 rows: ragged last tile
    ("2d7_b2", lambda: gi.convdiff(7, 2, 2.0)),                 # 49 rows: less than one slice
    ("3d40_b20", lambda: gi.convdiff(40, 3, 20.0)),
    # irregular patterns: every slice stored with explicit columns / a mix of both layouts
    ("2d40_rand", lambda: gi.convdiff_skew_perturbed(40, 2, 5.0, 3.0, 0.2, seed=3)),
    ("3d12_mixed", lambda: gi.convdiff_skew_perturbed(12, 3, 8.0, 2.0, 0.2, seed=4, rows_fraction=0.02)),
    # every slice diagonal-style, 8 offsets: per-slice metadata without explicit columns
    ("band8", lambda: banded(3001, (1, 2, 37, 300), seed=5)),
]

# expected storage: offsets per slice of the uniform layout (0 = per-slice metadata)
# and whether explicit columns are stored
LAYOUT = {"2d64_b10": (4, False), "3d17_b": (6, False), "2d7_b2": (4, False), "3d40_b20": (6, False),
          "2d40_rand": (0, True), "3d12_mixed": (0, True), "band8": (0, False)}


@pytest.fixture(scope="module", params=CASES, ids=[c[0] for c in CASES])
def case(request):
    A = request.param[1]()
    return A, gadi.System(A), oracle.OracleSystem(A)


def _dense_split16(osys, which):
    rp, col, val = osys.split(which)
    return rp, col, val.astype(np.float16)


def _csr_abs_mv(rp, col, val, x):
    n = len(rp) - 1
    y = np.zeros(n)
    for i in range(n):
        s = rp[i]
        e = rp[i + 1]
        y[i] = np.sum(np.abs(val[s:e]) * np.abs(x[col[s:e]]))
    return y


def _csr_mv(rp, col, val, x):
    import scipy.sparse as sp
    n = len(rp) - 1
    return sp.csr_matrix((val.astype(np.float64), col, rp), shape=(n, n)) @ x


def test_split_fp16_matches_rounded_oracle(case):
    A, g, o = case
    for which in ("H", "S"):
        rp, col, v16 = g.split_fp16(which)
        orp, ocol, oval = o.split(which)
        # the device pattern always carries the diagonal; compare entry by entry
        dev = {}
        for i in range(A.n):
            for k in range(rp[i], rp[i + 1]):
                dev[(i, int(col[k]))] = v16[k]
        for i in range(A.n):
            for k in range(orp[i], orp[i + 1]):
                key = (i, int(ocol[k]))
                assert np.float16(oval[k]).view(np.uint16) == np.float16(dev.get(key, 0.0)).view(np.uint16)
        assert set(k for k, v in dev.items() if v != 0) <= set((i, int(ocol[k])) for i in range(A.n)
                                                               for k in range(orp[i], orp[i + 1]))


def test_layout_kind(case, request):
    """Stencil matrices get the uniform diagonal layout, the others per-slice metadata."""
    A, g, o = case
    name = request.node.callspec.id
    lay = g.layout()
    w, expl = LAYOUT[name]
    assert lay["uniform_offsets"] == w
    assert (lay["explicit_entries"] > 0) == expl
    assert lay["nnz_off"] == sum(int(c != i) for i in range(A.n) for c in
                                 set(A.col[A.row_ptr[i]:A.row_ptr[i + 1]]) | set(_transpose_cols(A, i)))
    if w:
        assert lay["slots"] == w * lay["npad"] == lay["dia_slots"]


def _transpose_cols(A, i):
    if not hasattr(A, "_tcols"):
        cols = [[] for _ in range(A.n)]
        for r in range(A.n):
            for c in A.col[A.row_ptr[r]:A.row_ptr[r + 1]]:
                cols[c].append(r)
        A._tcols = cols
    return A._tcols[i]


def test_spmv_a64(case):
    A, g, o = case
    x = np.random.default_rng(11).uniform(-1, 1, A.n)
    xd = torch.from_numpy(x).cuda()
    yd = torch.empty_like(xd)
    g.spmv("A", xd, yd)
    torch.cuda.synchronize()
    y = yd.cpu().numpy()
    yref = o.spmv("A", x)
    bound = 8 * U64 * gi.csr_matvec(gi.Csr(A.n, A.row_ptr, A.col, np.abs(A.val)), np.abs(x))
    assert np.all(np.abs(y - yref) <= bound + 1e-300)


@pytest.mark.parametrize("alpha", [1e-3, 0.5, 10.0])
def test_spmv_h16(case, alpha):
    A, g, o = case
    rng = np.random.default_rng(12)
    x16 = rng.uniform(-1, 1, A.n).astype(np.float16)
    xd = torch.from_numpy(x16.view(np.int16)).cuda().view(torch.float16)
    yd = torch.empty_like(xd)
    g.spmv("H16", xd, yd, alpha)
    torch.cuda.synchronize()
    y = yd.cpu().numpy().astype(np.float64)
    rp, col, h16 = _dense_split16(o, "H")
    xv = x16.astype(np.float64)
    yref = alpha * xv + _csr_mv(rp, col, h16, xv)
    mag = alpha * np.abs(xv) + _csr_abs_mv(rp, col, h16.astype(np.float64), xv)
    assert np.all(np.abs(y - yref) <= (U16 + 8 * U32) * mag + 6e-8)


@pytest.mark.parametrize("alpha", [1e-3, 0.5, 10.0])
def test_spmv_s16(case, alpha):
    A, g, o = case
    rng = np.random.default_rng(13)
    x16 = rng.uniform(-1, 1, A.n).astype(np.float16)
    xd = torch.from_numpy(x16.view(np.int16)).cuda().view(torch.float16)
    yd = torch.empty_like(xd)
    g.spmv("S16", xd, yd, alpha)
    torch.cuda.synchronize()
    y = yd.cpu().numpy().astype(np.float64)
    rp, col, s16 = _dense_split16(o, "S")
    xv = x16.astype(np.float64)
    yref = xv + _csr_mv(rp, col, s16, xv) / alpha
    mag = np.abs(xv) + _csr_abs_mv(rp, col, s16.astype(np.float64), xv) / alpha
    rel = np.abs(y - yref) / np.maximum(mag, 1e-30)
    # y rounds once to half; the float sum carries <= 9 roundings of 2^-24, plus 1/alpha in float
    assert np.all(np.abs(y - yref) <= (U16 + 10 * U32) * mag + 6e-8), rel.max()


def test_features_match_oracle(case):
    A, g, o = case
    if not A.grid:
        pytest.skip("features describe convection-diffusion grids")
    f = g.features(A.dim, A.grid, A.beta)
    fo = oracle.features(A, o.gershgorin())
    assert np.allclose(f, fo, rtol=2e-7, atol=1e-7)


def _ref_solution(o, b):
    r = o.gadi(b, 0.5, 0.5, tol=1e-13, eps_h=1e-10, eps_s=1e-10)
    assert r["status"] == "ok"
    return r["x"]


def parity_tol(A, b, xref, target=1e-8, ref_tol=1e-13):
    """Outer tolerance that makes relative solution error <= target provable.

    ||x - x_ref|| <= (||r|| + ||r_ref||) / sigma_min(A) and sigma_min(A) >= lambda_min(H)
    because A is positive real; lambda_min(H) is the closed form of the splitting.
    Returns min(1e-10, the largest tol meeting the target)."""
    from oracle import dense as od
    if A.grid:
        lmin = od.convdiff_eigs_H(A.grid, A.dim)[0]
    else:
        # Gershgorin: lambda_min(H) >= min_i (H_ii - sum_j |H_ij|), positive for these matrices
        lmin = oracle.OracleSystem(A).gershgorin()[0]
        assert lmin > 0
    t = target * lmin * np.linalg.norm(xref) / np.linalg.norm(b) - ref_tol
    return min(1e-10, 0.9 * t)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
def test_solve_parity(case, prec):
    A, g, o = case
    xs, b = gi.rhs_for(A, "uniform", 0)
    xref = _ref_solution(o, b)
    tol = parity_tol(A, b, xref)
    assert tol >= 1e-12
    eps = 1e-6 if prec == "fp64" else None
    x, info = g.solve(b, 0.5, 0.5, tol=tol, prec=prec, eps_inner=eps)
    assert info["status"] == gadi.OK, info
    # FP64 residual recomputed on the CPU by the oracle
    rel = np.linalg.norm(b - o.spmv("A", x)) / np.linalg.norm(b)
    assert rel <= tol * 1.0000001, (rel, info)
    err = np.linalg.norm(x - xref) / np.linalg.norm(xref)
    assert err <= 1e-8, (err, tol, info)


def test_fp64_sweeps_match_oracle(case):
    """Same algorithm in the same precision: outer sweep counts agree within 2."""
    A, g, o = case
    xs, b = gi.rhs_for(A, "ones")
    ro = o.gadi(b, 0.5, 0.5, tol=1e-10, eps_h=1e-6, eps_s=1e-6)
    x, info = g.solve(b, 0.5, 0.5, tol=1e-10, prec="fp64", eps_inner=1e-6)
    assert info["status"] == gadi.OK
    assert abs(info["outer_sweeps"] - ro["sweeps"]) <= 2, (info, ro["sweeps"])
    assert abs(info["inner_H"] - ro["inner_h"]) <= 0.02 * ro["inner_h"] + 5
    assert np.linalg.norm(x - ro["x"]) <= 1e-8 * np.linalg.norm(ro["x"])


def test_history_and_warm_start():
    A = gi.convdiff(32, 2, 10.0)
    g = gadi.System(A)
    xs, b = gi.rhs_for(A)
    x1, i1 = g.solve(b, 0.5, 0.5, tol=1e-4, history=True)
    h = g.history
    assert len(h) == i1["outer_sweeps"] + 1 and h[0] == 1.0 and h[-1] <= 1e-4
    assert np.all(np.isfinite(h))
    x2, i2 = g.solve(b, 0.5, 0.5, tol=1e-6, x0=x1)
    o = oracle.OracleSystem(A)
    r1 = np.linalg.norm(b - o.spmv("A", x1))
    r2 = np.linalg.norm(b - o.spmv("A", x2))
    assert i2["status"] == gadi.OK and r2 <= 1.01e-6 * r1


def test_edge_cases():
    # one unknown: A = [4] (2-D, n = 1); the solve is exact after one sweep up to inner tolerance
    A = gi.convdiff(1, 2, 3.0)
    g = gadi.System(A)
    x, info = g.solve(np.array([8.0]), 0.5, 0.5, tol=1e-12, prec="fp64", eps_inner=1e-12)
    assert info["status"] == gadi.OK and abs(x[0] - 2.0) <= 1e-12
    # zero right-hand side: converged before any sweep, x untouched
    A = gi.convdiff(9, 3, 5.0)
    g = gadi.System(A)
    x, info = g.solve(np.zeros(A.n), 0.5, 0.5)
    assert info["status"] == gadi.OK and info["outer_sweeps"] == 0 and not np.any(x)
    # sweep limit: EMAXIT with the iterate returned
    xs, b = gi.rhs_for(A)
    x, info = g.solve(b, 0.5, 0.5, tol=1e-10, maxit_outer=3)
    assert info["status"] == gadi.EMAXIT and info["outer_sweeps"] == 3
    o = oracle.OracleSystem(A)
    assert np.linalg.norm(b - o.spmv("A", x)) < np.linalg.norm(b)
    # invalid parameters
    for al, om in ((0.0, 0.5), (-1.0, 0.5), (0.5, 2.0), (0.5, -0.1), (float("nan"), 0.5)):
        _, info = g.solve(b, al, om)
        assert info["status"] == gadi.EINVAL


def test_malformed_csr_rejected():
    bad = gi.Csr(3, np.array([0, 1, 2, 4], np.int32), np.array([0, 1, 2, 7], np.int32), np.ones(4))
    with pytest.raises(gadi.GadiError):
        gadi.System(bad)
    unsorted = gi.Csr(2, np.array([0, 2, 3], np.int32), np.array([1, 0, 1], np.int32), np.ones(3))
    with pytest.raises(gadi.GadiError):
        gadi.System(unsorted)


def test_device_pointers_and_stream():
    A = gi.convdiff(48, 2, 30.0)
    g = gadi.System(A)
    o = oracle.OracleSystem(A)
    xs, b = gi.rhs_for(A, "uniform", 5)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        bd = torch.from_numpy(b).cuda()
        x, info = g.solve(bd, 0.5, 0.5, tol=1e-10)
    torch.cuda.synchronize()
    assert info["status"] == gadi.OK
    xh = x.cpu().numpy()
    assert np.linalg.norm(b - o.spmv("A", xh)) <= 1.0000001e-10 * np.linalg.norm(b)


@pytest.mark.parametrize("alpha,omega", [(0.0215, 1.0), (10.0, 0.0), (0.464, 1.5), (0.1, 0.5)])
def test_fp16_regularisation_grid(alpha, omega):
    """Half-precision inner solves stay finite and converge across the (alpha, omega) grid."""
    A = gi.convdiff(16, 3, 20.0)
    g = gadi.System(A)
    o = oracle.OracleSystem(A)
    xs, b = gi.rhs_for(A, "uniform", 1)
    x, info = g.solve(b, alpha, omega, tol=1e-10, prec="fp16", maxit_outer=20000)
    assert info["status"] == gadi.OK, info
    assert np.linalg.norm(b - o.spmv("A", x)) <= 1.0000001e-10 * np.linalg.norm(b)


@pytest.mark.parametrize("form", [0, 1, 2, 3])
@pytest.mark.parametrize("prec", ["fp16", "h-d-s", "h-s-s", "fp8"])
def test_fp16_small_alpha_fails_cleanly_where_fp32_continues(prec, form, monkeypatch):
    """Too little regularisation: with alpha = 1e-3 the normal operator I - S^2/alpha^2 of the
    S-step exceeds the half range (||S||/alpha ~ 3.5e3 here).  The forms that apply it as one
    operator (0 and 1: (S/alpha)^2-sized intermediates) stop, in every mode that stores its Krylov
    vectors in half (fp16, h-d-s, h-s-s, fp8), with EOVERFLOW16 and a finite iterate (cf. the
    paper's Table 3d, where half-precision inner solves fail at the smallest alpha).  Craig's
    CGNE (forms 2 and 3) applies I + S/alpha and I - S/alpha separately, so its intermediates stay near
    ||S||/alpha, inside the half range: it runs into the sweep limit like single precision, with a
    finite iterate.  Single precision keeps reducing the residual."""
    monkeypatch.setenv("GADI_SOLVE_FORM", str(form))
    A = gi.convdiff(16, 3, 20.0)
    g = gadi.System(A)
    o = oracle.OracleSystem(A)
    xs, b = gi.rhs_for(A, "uniform", 1)
    x, info = g.solve(b, 1e-3, 0.5, tol=1e-10, prec=prec, maxit_outer=5, maxit_inner=500)
    assert g.solver_form() == form
    if form >= 2:
        assert info["status"] == gadi.EMAXIT and info["outer_sweeps"] == 5, info
    else:
        assert info["status"] == gadi.EOVERFLOW16, info
    assert np.all(np.isfinite(x))
    x, info = g.solve(b, 1e-3, 0.5, tol=1e-10, prec="fp32", maxit_outer=5, maxit_inner=500)
    assert info["status"] == gadi.EMAXIT and info["outer_sweeps"] == 5, info
    assert np.linalg.norm(b - o.spmv("A", x)) < np.linalg.norm(b)
