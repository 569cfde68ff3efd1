"""GPU tests of the batched (alpha, omega) sweep and the MLP predictor kernels.

The batched launch is checked against single-system solves through the same C
ABI (same algorithm, block-local instead of device-wide reductions) and
against the CPU oracle's residual; the MLP kernels are checked against the
float64 numpy MLP oracle, which is itself pinned by finite differences.
"""
import numpy as np
import pytest

import gadi_inputs as gi
import oracle
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2501_04229_amd as gadi  # noqa: E402

FAMILY = [(12, 2, 5.0), (30, 2, 80.0), (7, 3, (2.0, 9.0, 30.0)), (9, 3, 1.0), (20, 2, 300.0), (5, 3, 0.0)]
ALPHAS = [0.0215, 0.464, 2.0, 10.0]
OMEGAS = [1.0, 0.5, 0.0, 1.5]


@pytest.fixture(scope="module")
def family():
    out = []
    for i, (n, dim, beta) in enumerate(FAMILY):
        A = gi.convdiff(n, dim, beta)
        xs, b = gi.rhs_for(A, "uniform", 100 + i)
        out.append((A, b, gadi.System(A), oracle.OracleSystem(A)))
    return out


@pytest.mark.parametrize("prec", ["fp16", "fp64"])
def test_batched_matches_single_solves(family, prec, monkeypatch):
    """The batched kernel runs the Chronopoulos-Gear inner form; the single solves are pinned to
    the same form, so that failure statuses (the half overflow of I - (S/alpha)^2 at small alpha,
    which Craig's CGNE does not meet) agree trial by trial."""
    monkeypatch.setenv("GADI_SOLVE_FORM", "1")
    systems = [f[2] for f in family]
    bs = [f[1] for f in family]
    eps = 1e-6 if prec == "fp64" else None
    recs, xs = gadi.solve_batched(systems, bs, ALPHAS, OMEGAS, tol=1e-10, prec=prec, eps_inner=eps,
                                  maxit_outer=4000, want_x=True)
    for si, (A, b, g, o) in enumerate(family):
        for ti, (al, om) in enumerate(zip(ALPHAS, OMEGAS)):
            r = recs[si][ti]
            x1, i1 = g.solve(b, al, om, tol=1e-10, prec=prec, eps_inner=eps, maxit_outer=4000)
            assert r["status"] == i1["status"], (si, ti, r, i1)
            assert r["alpha"] == al and r["omega"] == om
            if i1["status"] == gadi.OK:
                # reduction order differs (block-local vs device-wide): counts agree closely
                assert abs(r["outer_sweeps"] - i1["outer_sweeps"]) <= max(2, 0.02 * i1["outer_sweeps"]), (si, ti)
                assert r["relres"] <= 1e-10
        # trial 0's solution: FP64 residual recomputed by the oracle
        if recs[si][0]["status"] == gadi.OK:
            assert np.linalg.norm(b - o.spmv("A", xs[si])) <= 1.0000001e-10 * np.linalg.norm(b)


def test_batched_is_reproducible_and_isolates_failures(family):
    systems = [f[2] for f in family]
    bs = [f[1] for f in family]
    alphas = [1e-3, 0.464]
    omegas = [0.5, 0.5]
    r1, x1 = gadi.solve_batched(systems, bs, alphas, omegas, tol=1e-10, prec="fp16", maxit_outer=300, want_x=True)
    r2, x2 = gadi.solve_batched(systems, bs, alphas, omegas, tol=1e-10, prec="fp16", maxit_outer=300, want_x=True)
    for si in range(len(systems)):
        for ti in range(2):
            a, b = r1[si][ti], r2[si][ti]
            for k in ("status", "outer_sweeps", "inner_H", "inner_S", "relres"):
                assert a[k] == b[k], (si, ti, k)
        assert np.array_equal(x1[si], x2[si])
        # the well-regularised trial converges whatever its neighbour trial does
        assert r1[si][1]["status"] == gadi.OK
        assert r1[si][0]["status"] in (gadi.OK, gadi.EOVERFLOW16, gadi.EMAXIT, gadi.EDIVERGED)


def test_batched_argument_checks(family):
    systems = [family[0][2]]
    bs = [family[0][1]]
    with pytest.raises(gadi.GadiError):
        gadi.solve_batched(systems, bs, [0.5] * 17, [0.5] * 17)
    with pytest.raises(gadi.GadiError):
        gadi.solve_batched(systems, bs, [0.0], [0.5])
    with pytest.raises(gadi.GadiError):
        gadi.solve_batched(systems, bs, [0.5], [2.0])


# ------------------------------------------------------------------ MLP
def _rand_problem(seed, B):
    rng = np.random.default_rng(seed)
    th = omlp.init(seed).astype(np.float32)
    th[512:576] = rng.normal(size=64).astype(np.float32) * 0.1
    X = rng.normal(size=(B, 8)).astype(np.float32)
    Y = rng.normal(size=(B, 2)).astype(np.float32)
    return th, X, Y


@pytest.mark.parametrize("B", [1, 7, 300])
def test_mlp_forward_matches_oracle(B):
    th, X, Y = _rand_problem(1, B)
    p = gadi.Predictor(seed=3)
    p.set_weights(th)
    p.set_norm(np.zeros(8), np.ones(8))
    y = p.forward(X)
    yref, _ = omlp.forward(th.astype(np.float64), X.astype(np.float64))
    assert np.allclose(y, yref, rtol=1e-5, atol=1e-5 * np.abs(yref).max())


@pytest.mark.parametrize("B", [1, 16, 256])
def test_mlp_gradient_matches_oracle(B):
    th, X, Y = _rand_problem(2, B)
    p = gadi.Predictor()
    p.set_weights(th)
    L, g = p.loss_grad(X, Y)
    Lr, gr = omlp.loss_grad(th.astype(np.float64), X.astype(np.float64), Y.astype(np.float64))
    assert abs(L - Lr) <= 1e-5 * abs(Lr)
    assert np.linalg.norm(g - gr) <= 1e-4 * np.linalg.norm(gr)
    big = np.abs(gr) > 1e-3 * np.abs(gr).max()
    assert np.allclose(g[big], gr[big], rtol=1e-3)


def test_mlp_training_follows_oracle_adam():
    """A few full-batch Adam steps on the device track the float64 oracle's trajectory."""
    th, X, Y = _rand_problem(4, 64)
    p = gadi.Predictor()
    p.set_weights(th)
    losses = p.train(X, Y, epochs=5, lr=1e-3)
    mu, sd = omlp.standardise_fit(X.astype(np.float64))
    Xs = (X - mu) / sd
    t = th.astype(np.float64)
    m = np.zeros_like(t)
    v = np.zeros_like(t)
    ref = []
    for k in range(1, 6):
        L, g = omlp.loss_grad(t, Xs, Y.astype(np.float64))
        ref.append(L)
        t, m, v = omlp.adam_step(t, g, m, v, k, lr=1e-3)
    assert np.allclose(losses, ref, rtol=1e-4)
    assert np.allclose(p.weights(), t, rtol=1e-3, atol=1e-5)


def test_mlp_training_fits_and_predicts_in_range():
    rng = np.random.default_rng(5)
    X = rng.normal(size=(200, 8)).astype(np.float32) * 3 + 1
    Y = np.stack([np.tanh(X[:, 0] / 3) - 1.0, 0.5 + 0.2 * np.tanh(X[:, 1] / 3)], axis=1).astype(np.float32)
    p = gadi.Predictor(seed=1)
    losses = p.train(X, Y, epochs=1500, lr=3e-3)
    assert losses[-1] < 0.02 * losses[0]
    # alpha = 10^(y0 + (f4 + f5) / 2): the network's output on the alpha_ref scale;
    # take a sample whose alpha lies inside the clamp range [1e-3, 10]
    la = Y[:, 0] + 0.5 * (X[:, 4] + X[:, 5])
    i = int(np.flatnonzero((la > -2.5) & (la < 0.5))[0])
    a, w = p.predict(X[i])
    assert 1e-3 <= a <= 10.0 and 0.0 <= w <= 1.99
    y0 = np.log10(a) - 0.5 * (float(X[i, 4]) + float(X[i, 5]))
    assert abs(y0 - Y[i, 0]) < 0.15 and abs(w - Y[i, 1]) < 0.1


def test_mlp_inputs_clamped_to_training_range():
    """Raw features outside [lo, hi] give the prediction of the clamped features."""
    th, X, Y = _rand_problem(6, 4)
    p = gadi.Predictor()
    p.set_weights(th)
    p.set_norm(np.zeros(8), np.ones(8))
    lo, hi = -np.ones(8, np.float32), np.ones(8, np.float32)
    p.set_bounds(lo, hi)
    Xo = (X * 5).astype(np.float32)
    y = p.forward(Xo)
    yref, _ = omlp.forward(th.astype(np.float64), np.clip(Xo, lo, hi).astype(np.float64))
    assert np.allclose(y, yref, rtol=1e-5, atol=1e-5 * np.abs(yref).max())
    with pytest.raises(gadi.GadiError):
        p.set_bounds(hi, lo)


def test_trained_predictor_stays_in_grid_range():
    """The committed weights predict alpha and omega inside the trial grid's span for the bench systems."""
    from paper_2501_04229_amd import predictor as pr
    p = pr.load()
    for n, dim, beta in ((128, 3, 20.0), (64, 2, 10.0), (40, 3, 300.0)):
        A = gi.convdiff(n, dim, beta)
        g = gadi.System(A)
        a, w = pr.predict(p, g, A)
        assert 1e-3 <= a <= 10.0 and 0.0 <= w <= 1.99


def _constant_predictor(y0, omega):
    """A network whose output is the constant (y0, omega): zero weights, output bias only."""
    th = np.zeros(4866, np.float32)
    th[-2] = y0
    th[-1] = omega
    p = gadi.Predictor()
    p.set_weights(th)
    p.set_norm(np.zeros(8), np.ones(8))
    return p


def test_solve_auto_keeps_a_good_prediction():
    """The trained predictor on a fresh system: the prediction is kept and the FP64 residual,
    recomputed by the oracle, meets the tolerance."""
    from paper_2501_04229_amd import predictor as pr
    A = gi.convdiff(20, 3, 30.0)
    g = gadi.System(A)
    o = oracle.OracleSystem(A)
    xs, b = gi.rhs_for(A, "uniform", 7)
    x, info, used = pr.solve_auto(g, A, b, pr.load(), tol=1e-10)
    assert used == "mlp" and info["fell_back"] == 0 and info["status"] == gadi.OK, info
    assert np.linalg.norm(b - o.spmv("A", x)) <= 1.0000001e-10 * np.linalg.norm(b)
    assert info["launches"] >= 1


def test_solve_auto_falls_back_when_the_prediction_fails():
    """alpha clamped to 1e-3 overflows the half-precision S-step on this system: the guard
    replaces the prediction by the default (0.5, 0.5) from x = 0, which converges."""
    from paper_2501_04229_amd import predictor as pr
    A = gi.convdiff(16, 3, 20.0)
    g = gadi.System(A)
    o = oracle.OracleSystem(A)
    xs, b = gi.rhs_for(A, "uniform", 1)
    p = _constant_predictor(-20.0, 0.5)
    a, w = pr.predict(p, g, A)
    assert a == 1e-3 and w == 0.5
    x, info, used = pr.solve_auto(g, A, b, p, tol=1e-10)
    assert used == "default" and info["fell_back"] == 1 and info["status"] == gadi.OK, info
    assert np.linalg.norm(b - o.spmv("A", x)) <= 1.0000001e-10 * np.linalg.norm(b)
    x1, i1 = g.solve(b, 0.5, 0.5, tol=1e-10)
    # the default run is the whole solve after the failed probe
    assert info["outer_sweeps"] - i1["outer_sweeps"] <= 32


def test_solve_auto_rejects_a_prediction_slower_than_the_default():
    """A constant prediction that converges, but needs more than twice the default's work (an
    alpha far off the optimum of the alpha U-curve, picked among a few candidates by measuring
    them).  The old guard kept any prediction that reached the tolerance within the sweep budget;
    the default judges it now: the prediction may spend the work of a default solve, has not
    converged by then, and the default finishes from its iterate -- the whole solve costs less
    work than the prediction alone."""
    from paper_2501_04229_amd import predictor as pr
    A = gi.convdiff(16, 3, 20.0)
    g = gadi.System(A)
    o = oracle.OracleSystem(A)
    xs, b = gi.rhs_for(A, "uniform", 2)
    f = g.features(A.dim, A.grid, A.beta)
    _, fast = g.solve(b, 0.5, 0.5, tol=1e-10)
    assert fast["status"] == gadi.OK
    slow = None
    for a_slow in (0.1, 0.05, 0.03, 8.0):
        _, rec = g.solve(b, a_slow, 0.5, tol=1e-10)
        if rec["status"] == gadi.OK and pr.work(rec) > 2 * pr.work(fast):
            slow = rec
            break
    assert slow is not None, "no slower converging alpha among the candidates"
    p = _constant_predictor(np.log10(a_slow) - pr.log_alpha_ref(f), 0.5)
    a, w = pr.predict(p, g, A)
    assert abs(a - a_slow) < 1e-3 * a_slow and w == 0.5
    x, info, used = pr.solve_auto(g, A, b, p, tol=1e-10, judge="measure")
    assert used == "default" and info["fell_back"] == 1 and info["status"] == gadi.OK, info
    assert np.linalg.norm(b - o.spmv("A", x)) <= 1.0000001e-10 * np.linalg.norm(b)
    # the prediction spent at most the default's work, then the default finished from its iterate
    assert info["guard"]["judge_work"] == pr.work(fast)
    assert pr.work(info) < pr.work(slow), (info, slow)
    # the judge is measured once per handle and reused
    assert info["guard_seconds"] > 0
    x, info2, used2 = pr.solve_auto(g, A, b, p, tol=1e-10, judge="measure")
    assert used2 == "default" and info2["guard_seconds"] == 0.0


def test_pruned_trials_carry_their_own_status(family):
    """With prune_dominated, a trial whose work passes that of a converged trial of the same
    system stops with EPRUNED (not EMAXIT): its work is above the least converged work of its
    system, and every system's cheapest converged trial is the one an unpruned launch finds."""
    from paper_2501_04229_amd import predictor as pr
    systems = [f[2] for f in family]
    bs = [f[1] for f in family]
    alphas = [0.0215, 0.464, 2.0, 10.0, 0.1, 1.0, 5.0, 0.05]
    omegas = [1.0, 0.5, 0.0, 1.5, 0.5, 1.0, 0.5, 0.0]
    pruned, _ = gadi.solve_batched(systems, bs, alphas, omegas, tol=1e-10, prec="fp16", maxit_outer=4000,
                                   prune=True)
    full, _ = gadi.solve_batched(systems, bs, alphas, omegas, tol=1e-10, prec="fp16", maxit_outer=4000,
                                 prune=False)
    n_pruned = 0
    for si in range(len(systems)):
        ok_full = [pr.work(r) for r in full[si] if r["status"] == gadi.OK]
        ok_pruned = [pr.work(r) for r in pruned[si] if r["status"] == gadi.OK]
        if not ok_full:
            continue
        # the cheapest converged trial survives pruning, with the same work
        assert min(ok_pruned) == min(ok_full), (si, ok_pruned, ok_full)
        assert all(r["status"] != gadi.EPRUNED for r in full[si])
        for r in pruned[si]:
            if r["status"] == gadi.EPRUNED:
                n_pruned += 1
                assert pr.work(r) > min(ok_pruned), (si, r)
    assert n_pruned > 0
