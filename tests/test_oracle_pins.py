"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every check here runs on the CPU.  The oracle is compared with values that do
not come from the oracle itself: the two written forms of the GADI iteration
(Section 2.1), Theorem 1's iteration matrix, closed-form spectra of the
convection-diffusion splitting, the Bai-Golub-Ng HSS bound, a DST-I spectral
solution for beta = 0, dense direct solves and the manufactured solution of
Section 4.1, and the paper's Table 1 constants.
"""
import math
import os

import numpy as np
import pytest

import gadi_inputs as gi
import oracle
from oracle import dense as od

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

TINY = [
    (8, 2, 10.0),
    (5, 3, (3.0, 7.0, 11.0)),
    (6, 3, 10.0),
]


def _sys(n, dim, beta):
    A = gi.convdiff(n, dim, beta)
    return A, od.dense(A)


# ---------------------------------------------------------------- generator
@pytest.mark.parametrize("n,dim", [(1, 2), (2, 2), (7, 2), (64, 2), (1, 3), (3, 3), (17, 3)])
def test_generator_matches_kronecker_definition(n, dim):
    """The CSR generator reproduces the Kronecker-sum form of Section 4.1."""
    import scipy.sparse as sp
    beta = (2.5, 4.0, 9.0)[:dim]
    A = gi.convdiff(n, dim, beta)
    assert A.nnz == gi.convdiff_nnz(n, dim)
    r = [b / (2 * (n + 1)) for b in beta]

    def T(diag, ra):
        return sp.diags([(-1 - ra) * np.ones(n - 1), diag * np.ones(n), (-1 + ra) * np.ones(n - 1)],
                        [-1, 0, 1], shape=(n, n))
    I = sp.identity(n)
    if dim == 2:
        K = sp.kron(T(4.0, r[0]), I) + sp.kron(I, T(0.0, r[1]))
    else:
        K = (sp.kron(sp.kron(T(6.0, r[0]), I), I) + sp.kron(sp.kron(I, T(0.0, r[1])), I)
             + sp.kron(sp.kron(I, I), T(0.0, r[2])))
    assert abs(A.to_scipy() - K).max() == 0.0
    # sorted, unique columns per row
    for i in range(min(A.n, 200)):
        c = A.col[A.row_ptr[i]:A.row_ptr[i + 1]]
        assert np.all(np.diff(c) > 0)


def test_generator_manufactured_rhs():
    A = gi.convdiff(9, 3, 5.0)
    xs, b = gi.rhs_for(A, "ones")
    assert np.allclose(b, od.dense(A) @ np.ones(A.n), rtol=0, atol=1e-14)


# ---------------------------------------------------------------- P1
@pytest.mark.parametrize("n,dim,beta", TINY)
@pytest.mark.parametrize("alpha,omega", [(0.1, 0.0), (0.5, 0.5), (2.0, 1.5), (0.05, 1.0)])
def test_p1_correction_form_equals_gadi_equation(n, dim, beta, alpha, omega):
    """Algorithm 1 with exact inner solves reproduces the two-half-step GADI equation."""
    A, Ad = _sys(n, dim, beta)
    b = Ad @ np.random.default_rng(5).uniform(-1, 1, A.n)
    st = od.gadi_stationary(Ad, b, alpha, omega, 12)
    co, _ = od.gadi_correction(Ad, b, alpha, omega, sweeps=12)
    for xs, xc in zip(st, co):
        assert np.linalg.norm(xs - xc) <= 1e-12 * max(1.0, np.linalg.norm(xs))


@pytest.mark.parametrize("n,dim,beta", TINY)
@pytest.mark.parametrize("alpha,omega", [(0.5, 0.5), (0.2, 1.0), (3.0, 0.0)])
def test_p1_c_oracle_follows_exact_iterates(n, dim, beta, alpha, omega):
    """The C oracle with tight inner tolerances matches the exact-inner iterates sweep by sweep."""
    A, Ad = _sys(n, dim, beta)
    b = Ad @ np.ones(A.n)
    co, _ = od.gadi_correction(Ad, b, alpha, omega, sweeps=8)
    s = oracle.OracleSystem(A)
    for k in (1, 2, 5, 8):
        r = s.gadi(b, alpha, omega, tol=0.0, eps_h=1e-14, eps_s=1e-14, maxit_out=k, maxit_in=10 * A.n)
        assert r["sweeps"] == k and r["status"] == "emaxit"
        assert np.linalg.norm(r["x"] - co[k]) <= 1e-11 * np.linalg.norm(co[k])


def test_p1_sweep_counts_match_exact_form():
    A, Ad = _sys(8, 2, 10.0)
    b = Ad @ np.ones(A.n)
    _, res = od.gadi_correction(Ad, b, 0.5, 0.5, tol=1e-10)
    r = oracle.OracleSystem(A).gadi(b, 0.5, 0.5, tol=1e-10, eps_h=1e-13, eps_s=1e-13)
    assert r["status"] == "ok"
    assert abs(r["sweeps"] - (len(res) - 1)) <= 1


# ---------------------------------------------------------------- P2
@pytest.mark.parametrize("n,dim,beta", TINY)
def test_p2_theorem1_matrix_and_contraction(n, dim, beta):
    """Theorem 1's T equals the correction-form error propagator and rho(T) < 1."""
    _, Ad = _sys(n, dim, beta)
    for alpha in (0.01, 0.1, 1.0, 10.0):
        for omega in (0.0, 0.5, 1.0, 1.5, 1.9):
            T = od.iteration_matrix(Ad, alpha, omega)
            Tc = od.iteration_matrix_correction(Ad, alpha, omega)
            assert np.abs(T - Tc).max() <= 1e-11 * max(1.0, np.abs(T).max())
            assert od.spectral_radius(T) < 1.0


def test_p2_observed_rate_matches_spectral_radius():
    """The oracle's asymptotic residual ratio approaches rho(T)."""
    A, Ad = _sys(6, 3, 10.0)
    rho = od.spectral_radius(od.iteration_matrix(Ad, 0.5, 0.5))
    b = Ad @ np.random.default_rng(3).uniform(-1, 1, A.n)
    r = oracle.OracleSystem(A).gadi(b, 0.5, 0.5, tol=1e-13, eps_h=1e-14, eps_s=1e-14,
                                    maxit_in=10 * A.n, hist_len=2000)
    h = r["hist"]
    k1 = int(np.argmax(h < 1e-5))
    k2 = int(np.argmax(h < 1e-11))
    assert k2 > k1 + 10
    rate = (h[k2] / h[k1]) ** (1.0 / (k2 - k1))
    assert abs(rate - rho) <= 0.05 * rho


# ---------------------------------------------------------------- P3
@pytest.mark.parametrize("n,dim", [(6, 3), (8, 2), (5, 3)])
@pytest.mark.parametrize("alpha", [0.05, 0.5, 2.0])
def test_p3_hss_bound(n, dim, alpha):
    """omega = 0 is HSS: rho(T) <= max |alpha - l| / (alpha + l) over eig(H)."""
    _, Ad = _sys(n, dim, 10.0)
    rho = od.spectral_radius(od.iteration_matrix(Ad, alpha, 0.0))
    assert rho <= od.hss_contraction_bound(n, dim, alpha) + 1e-12


# ---------------------------------------------------------------- P4
@pytest.mark.parametrize("n,dim", [(6, 3), (9, 2)])
@pytest.mark.parametrize("alpha,omega", [(0.5, 0.5), (0.1, 1.2)])
def test_p4_beta0_spectral_iterates(n, dim, alpha, omega):
    """beta = 0: S = 0 and the iteration acts on DST-I modes with factor 1 - (2-omega) l/(alpha+l)."""
    A = gi.convdiff(n, dim, 0.0)
    xs = np.random.default_rng(7).uniform(-1, 1, A.n)
    b = gi.csr_matvec(A, xs)
    Q1 = od.dst1_modes(n, dim)
    Q = Q1
    for _ in range(dim - 1):
        Q = np.kron(Q, Q1)
    lam1 = 2.0 - 2.0 * np.cos(np.arange(1, n + 1) * np.pi / (n + 1))
    lam = lam1
    for _ in range(dim - 1):
        lam = np.add.outer(lam, lam1).ravel()
    mu = 1.0 - (2.0 - omega) * lam / (alpha + lam)
    c = Q.T @ xs
    s = oracle.OracleSystem(A)
    for k in (1, 3, 10):
        xk = xs - Q @ (mu ** k * c)
        r = s.gadi(b, alpha, omega, tol=0.0, eps_h=1e-15, eps_s=1e-15, maxit_out=k, maxit_in=10 * A.n)
        assert np.linalg.norm(r["x"] - xk) <= 1e-11 * np.linalg.norm(xk)


# ---------------------------------------------------------------- P5
@pytest.mark.parametrize("n,dim,beta", TINY + [(12, 2, 50.0)])
def test_p5_solution_matches_direct_solve(n, dim, beta):
    A, Ad = _sys(n, dim, beta)
    b = Ad @ np.ones(A.n)
    r = oracle.OracleSystem(A).gadi(b, 0.5, 0.5, tol=1e-12)
    assert r["status"] == "ok" and r["relres"] <= 1e-12
    xd = np.linalg.solve(Ad, b)
    assert np.linalg.norm(r["x"] - xd) <= 1e-9 * np.linalg.norm(xd)
    assert np.linalg.norm(r["x"] - 1.0) <= 1e-9 * math.sqrt(A.n)


def test_p5_config1_forward_error():
    """2-D n = 64, beta = 10, (0.5, 0.5), inner 1e-6, tol 1e-10: x ~ 1 to the forward-error bound."""
    A = gi.convdiff(64, 2, 10.0)
    xs, b = gi.rhs_for(A, "ones")
    r = oracle.OracleSystem(A).gadi(b, 0.5, 0.5, tol=1e-10, eps_h=1e-6, eps_s=1e-6)
    assert r["status"] == "ok" and r["relres"] <= 1e-10
    # ||x - x*|| / ||x*|| <= tol ||r0|| / (sigma_min(A) ||x*||), sigma_min >= lambda_min(H)
    lmin = od.convdiff_eigs_H(64, 2)[0]
    bound = 1e-10 * np.linalg.norm(b) / (lmin * np.linalg.norm(xs))
    assert np.linalg.norm(r["x"] - xs) / np.linalg.norm(xs) <= bound


# ---------------------------------------------------------------- P6
@pytest.mark.parametrize("n,dim,beta", TINY)
def test_p6_splitting_invariants(n, dim, beta):
    A, Ad = _sys(n, dim, beta)
    s = oracle.OracleSystem(A)
    assert s.split_ok
    H = od.dense(gi.Csr(A.n, *s.split("H")))
    S = od.dense(gi.Csr(A.n, *s.split("S")))
    assert np.array_equal(H, H.T) and np.array_equal(S, -S.T)
    assert np.abs(H + S - Ad).max() <= 4 * np.finfo(float).eps * np.abs(Ad).max()
    x = np.random.default_rng(1).uniform(-1, 1, A.n)
    assert abs(x @ S @ x) <= 1e-14 * (x @ x) * np.abs(S).sum()
    for alpha in (1e-3, 0.5):
        np.linalg.cholesky(alpha * np.eye(A.n) + H)
        assert np.linalg.eigvalsh(alpha * np.eye(A.n) + H)[0] >= alpha - 1e-12
        sv = np.linalg.svd(alpha * np.eye(A.n) + S, compute_uv=False)
        svS = np.linalg.svd(S, compute_uv=False)
        assert np.allclose(np.sort(sv), np.sort(np.sqrt(alpha ** 2 + svS ** 2)), rtol=1e-12, atol=1e-13)


def test_p6_nonsymmetric_pattern_split():
    """A general CSR with a non-symmetric pattern: the splitting lives on the union pattern."""
    rp = np.array([0, 2, 3, 5], dtype=np.int32)
    col = np.array([0, 2, 1, 0, 2], dtype=np.int32)
    val = np.array([4.0, -1.5, 3.0, 0.5, 5.0])
    A = gi.Csr(3, rp, col, val)
    s = oracle.OracleSystem(A)
    assert s.split_ok
    Ad = od.dense(A)
    H = od.dense(gi.Csr(3, *s.split("H")))
    S = od.dense(gi.Csr(3, *s.split("S")))
    assert np.array_equal(H, (Ad + Ad.T) / 2) and np.array_equal(S, (Ad - Ad.T) / 2)


def test_p6_rejects_malformed_csr():
    with pytest.raises(ValueError):
        oracle.OracleSystem(gi.Csr(2, np.array([0, 1, 3], np.int32), np.array([0, 1, 5], np.int32),
                                   np.ones(3)))
    with pytest.raises(ValueError):
        oracle.OracleSystem(gi.Csr(2, np.array([0, 2, 2], np.int32), np.array([1, 0], np.int32),
                                   np.ones(2)))


# ---------------------------------------------------------------- P7
@pytest.mark.parametrize("n,dim,beta", [(8, 2, 10.0), (5, 3, 4.0), (7, 3, 30.0)])
def test_p7_closed_form_spectra_and_gershgorin(n, dim, beta):
    A, Ad = _sys(n, dim, beta)
    H, S = od.hss(Ad)
    lh = np.linalg.eigvalsh(H)
    assert np.allclose(lh, od.convdiff_eigs_H(n, dim), atol=1e-12)
    ls = np.linalg.eigvals(S)
    assert np.abs(ls.real).max() <= 1e-12
    assert np.allclose(np.sort(ls.imag), od.convdiff_eigs_S_imag(n, dim, beta), atol=1e-12)
    g = oracle.OracleSystem(A).gershgorin()
    r = beta / (2.0 * (n + 1))
    assert g[0] == 0.0 and g[1] == 4.0 * dim
    assert math.isclose(g[2], 2 * dim * r, rel_tol=1e-14) and math.isclose(g[3], dim * r, rel_tol=1e-14)
    assert g[0] <= lh[0] and lh[-1] <= g[1]
    assert np.abs(ls).max() <= g[2] + 1e-12


# ---------------------------------------------------------------- P8
@pytest.mark.parametrize("n,dim,beta,alpha", [(10, 3, 20.0, 0.5), (32, 2, 10.0, 0.05), (8, 3, 200.0, 0.1)])
def test_p8_inner_solvers(n, dim, beta, alpha):
    """One sweep: inner counts obey the CG bound; the correction equals the exact two solves."""
    A, Ad = _sys(n, dim, beta)
    b = Ad @ np.ones(A.n)
    eps = 1e-8
    r = oracle.OracleSystem(A).gadi(b, alpha, 0.5, tol=0.0, eps_h=eps, eps_s=eps, maxit_out=1)
    lh = od.convdiff_eigs_H(n, dim)
    kh = (alpha + lh[-1]) / (alpha + lh[0])
    sig = np.abs(od.convdiff_eigs_S_imag(n, dim, beta)).max()
    ks = (alpha ** 2 + sig ** 2) / alpha ** 2
    assert r["inner_h"] <= math.ceil(0.5 * math.sqrt(kh) * math.log(2 / eps)) + 1
    assert r["inner_s"] <= math.ceil(0.5 * math.sqrt(ks) * math.log(2 / eps)) + 1
    H, S = od.hss(Ad)
    I = np.eye(A.n)
    z = np.linalg.solve(alpha * I + H, b)
    y = np.linalg.solve(alpha * I + S, 1.5 * alpha * z)
    # inner relative residuals <= eps, amplified by the condition numbers
    assert np.linalg.norm(r["x"] - y) <= 10 * eps * (math.sqrt(kh) + math.sqrt(ks)) * np.linalg.norm(y) * 10


# ---------------------------------------------------------------- P11 / golden
def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def test_golden_precision_table():
    """Table 1 unit roundoffs equal the IEEE formats numpy implements."""
    rows = {r[0]: r for r in _read_golden("precision_table.txt")}
    for name, dt in (("half", np.float16), ("single", np.float32), ("double", np.float64)):
        fi = np.finfo(dt)
        u = float(fi.eps) / 2.0
        assert int(rows[name][1]) == fi.bits
        assert math.log2(u) == int(rows[name][2])
        assert abs(u - float(rows[name][3])) <= 0.05 * u
        assert abs(math.log10(float(fi.max)) - int(rows[name][4])) < 0.6


def test_golden_alpha_effects_is_u_shaped_and_oracle_agrees():
    """Table 'alpha-effects' is U-shaped in alpha; the FP64 oracle shows the same shape in sweeps."""
    rows = [r for r in _read_golden("alpha_effects.txt") if r[2] != "-"]
    steps = np.array([int(r[2]) for r in rows])
    k = int(np.argmin(steps))
    assert 0 < k < len(steps) - 1 and float(rows[k][0]) == 0.5
    A = gi.convdiff(12, 3, 1.0)
    xs, b = gi.rhs_for(A)
    s = oracle.OracleSystem(A)
    alphas = [0.02, 0.1, 0.5, 2.0, 10.0]
    sw = [s.gadi(b, a, 0.5, tol=1e-8, eps_h=1e-8, eps_s=1e-8)["sweeps"] for a in alphas]
    j = int(np.argmin(sw))
    assert 0 < j < len(alphas) - 1
    assert sw[0] > 2 * sw[j] and sw[-1] > 2 * sw[j]


def test_oracle_rejects_bad_parameters():
    A = gi.convdiff(4, 2, 1.0)
    s = oracle.OracleSystem(A)
    b = np.ones(A.n)
    assert s.gadi(b, 0.0, 0.5)["status"] == "einval"
    assert s.gadi(b, 0.5, 2.0)["status"] == "einval"
    assert s.gadi(b, -1.0, 0.5)["status"] == "einval"


def test_oracle_zero_rhs_and_warm_start():
    A = gi.convdiff(6, 2, 3.0)
    s = oracle.OracleSystem(A)
    r = s.gadi(np.zeros(A.n), 0.5, 0.5)
    assert r["status"] == "ok" and r["sweeps"] == 0 and not np.any(r["x"])
    xs, b = gi.rhs_for(A)
    r1 = s.gadi(b, 0.5, 0.5, tol=1e-6)
    r2 = s.gadi(b, 0.5, 0.5, tol=1e-4, x0=r1["x"])
    res1 = np.linalg.norm(b - s.spmv("A", r1["x"]))
    res2 = np.linalg.norm(b - s.spmv("A", r2["x"]))
    assert r2["status"] == "ok" and r2["sweeps"] > 0 and res2 <= 1e-4 * res1


def test_oracle_divergence_flag():
    """omega close to 2 with a tiny alpha on a coarse inner solve still reports a status, never hangs."""
    A = gi.convdiff(6, 2, 3.0)
    s = oracle.OracleSystem(A)
    xs, b = gi.rhs_for(A)
    r = s.gadi(b, 0.5, 0.5, tol=1e-10, maxit_out=3)
    assert r["status"] == "emaxit" and r["sweeps"] == 3


@pytest.mark.parametrize("plant", [1, 2])
def test_pins_catch_planted_oracle_mistakes(plant):
    """A deliberately wrong oracle build (sign flip in the CGNE back-substitution,
    or a wrong S-step scale) fails the sweep-by-sweep exact-iterate pin."""
    A, Ad = _sys(5, 3, (3.0, 7.0, 11.0))
    b = Ad @ np.ones(A.n)
    co, _ = od.gadi_correction(Ad, b, 0.5, 0.5, sweeps=2)
    bad = oracle.OracleSystem(A, plant=plant)
    r = bad.gadi(b, 0.5, 0.5, tol=0.0, eps_h=1e-14, eps_s=1e-14, maxit_out=2, maxit_in=10 * A.n)
    assert np.linalg.norm(r["x"] - co[2]) > 1e-3 * np.linalg.norm(co[2])


@pytest.mark.parametrize("n,dim,beta", [(5, 2, (10.0, 3.0)), (4, 3, (20.0, 1.0, 7.0)), (6, 2, 0.5),
                                        (3, 3, 100.0)])
def test_features_against_the_dense_matrix(n, dim, beta):
    """Every predictor feature against the assembled matrix itself (no closed form reused):
    lambda_min(H) from eigvalsh of the dense (A + A^T)/2, the cell Peclet number max_a beta_a h / 2
    as the largest |entry| of the dense (A - A^T)/2 (the skew entries are +-r_a), and the
    Gershgorin quantities from dense row sums.  A wrong mesh width (h = 1/n), a wrong factor in
    the Peclet number or a wrong eigenvalue formula fails."""
    A = gi.convdiff(n, dim, beta)
    D = np.zeros((A.n, A.n))
    for i in range(A.n):
        for k in range(A.row_ptr[i], A.row_ptr[i + 1]):
            D[i, A.col[k]] += A.val[k]
    H = 0.5 * (D + D.T)
    S = 0.5 * (D - D.T)
    f = oracle.features(A)
    b = np.broadcast_to(np.asarray(beta, dtype=float), (dim,))
    assert f[0] == pytest.approx(np.log(n ** dim), abs=1e-14)
    assert f[1] == dim
    assert f[2] == pytest.approx(np.log10(b.mean()), abs=1e-14)
    assert 10 ** f[3] == pytest.approx(np.abs(S).max(), rel=1e-12)
    assert 10 ** f[4] == pytest.approx(np.linalg.eigvalsh(H)[0], rel=1e-9)
    off_h = np.abs(H - np.diag(np.diag(H))).sum(axis=1)
    assert 10 ** f[5] == pytest.approx((np.diag(H) + off_h).max(), rel=1e-12)
    rs = np.abs(S).sum(axis=1)
    assert 10 ** f[6] == pytest.approx(rs.max(), rel=1e-12)
    assert 10 ** f[7] == pytest.approx(rs.min(), rel=1e-12)
