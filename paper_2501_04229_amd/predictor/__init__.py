"""(alpha, omega) prediction for GADI-IR.

The paper predicts the splitting parameter from small systems of the same
structure (Section 3.3: a training set of near-optimal parameters found on
small systems, then a regression used on large ones).  Here the regression is
the 8 -> 64 -> 64 -> 2 MLP of libgadi, trained on the device, and the training
set comes from the batched (alpha, omega) sweep of libgadi on small
convection-diffusion systems.

Label of a system: the trial with the least solver work among the trials that
reached the tolerance, where work = inner_H + 2 inner_S + 5 sweeps counts the
phases of the persistent solve kernel with the fused inner solvers (a CG step
is one phase, a CGNE step two, and each sweep adds the residual, the CG start,
the two CGNE start phases and the update).  Each phase ends in a device-wide
reduction, and on the large systems the solve time is proportional to this
count.  Ties go to fewer outer sweeps, then to the larger alpha.

Targets are (log10(alpha / alpha_ref), omega) with alpha_ref =
sqrt(lambda_min(H) lambda_max(H)) from features 4 and 5 (the optimal HSS
parameter of the symmetric part alone), so the network learns a scale-free
correction and the size dependence of alpha comes from the closed-form
spectrum; libgadi applies alpha = alpha_ref 10^y0 at prediction time.

The default parameters (0.5, 0.5) are both the fallback and the judge:
`solve_auto` replaces a prediction by the default if its first sweeps fail, or
once it has spent the work a default solve needs without converging.
"""
from __future__ import annotations

import math
import os

import numpy as np

import paper_2501_04229_amd as gadi
from gadi_inputs import ALPHA_GRID, OMEGA_GRID

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "mlp_weights.npz")
DEFAULT = (0.5, 0.5)


def trial_grid():
    """The 16 (alpha, omega) trials: 4 log-spaced alphas x 4 omegas."""
    al = [a for a in ALPHA_GRID for _ in OMEGA_GRID]
    om = [w for _ in ALPHA_GRID for w in OMEGA_GRID]
    return al, om


def work(rec) -> float:
    """Phases of the fused solve kernel for a solve record."""
    return float(rec["inner_H"] + 2 * rec["inner_S"] + 5 * rec["outer_sweeps"])


def log_alpha_ref(f) -> float:
    """log10 sqrt(lambda_min(H) lambda_max(H)) from a feature vector."""
    return 0.5 * (float(f[4]) + float(f[5]))


def label(recs):
    """Index of the best converged trial of one system, or None."""
    best = None
    for t, r in enumerate(recs):
        if r["status"] != gadi.OK:
            continue
        key = (work(r), r["outer_sweeps"], -r["alpha"])
        if best is None or key < best[0]:
            best = (key, t)
    return None if best is None else best[1]


def refine_grid(best_alpha, best_omega):
    """16 trials around a system's best coarse trial: alpha times 8 factors in
    [1/4, 4] (geometric), omega moved by -0.25 and +0.25 (kept in [0, 1.9])."""
    facs = np.geomspace(0.25, 4.0, 8)
    al, om = [], []
    for dw in (-0.25, 0.25):
        for f in facs:
            al.append(float(min(max(best_alpha * f, 1e-3), 10.0)))
            om.append(float(min(max(best_omega + dw, 0.0), 1.9)))
    return al, om


def sweep_table(metas, rhs, prec="fp16", tol=1e-10, maxit_outer=5000, eps_inner=None, refine=True):
    """Batched sweep over `metas` (gadi_inputs.Csr with grid metadata).

    Stage 1 runs the 16-trial grid on every system; stage 2 (refine=True)
    searches a per-system grid around each system's best stage-1 trial, the
    way the paper narrows alpha on small systems before regressing it.
    Returns (records [nsys][16 or 32], features [nsys, 8])."""
    systems = [gadi.System(A) for A in metas]
    al, om = trial_grid()
    recs, _ = gadi.solve_batched(systems, rhs, al, om, tol=tol, prec=prec, eps_inner=eps_inner,
                                 maxit_outer=maxit_outer, prune=True)
    if refine:
        idx = [s for s in range(len(systems)) if label(recs[s]) is not None]
        if idx:
            grids = [refine_grid(recs[s][label(recs[s])]["alpha"], recs[s][label(recs[s])]["omega"]) for s in idx]
            r2, _ = gadi.solve_batched([systems[s] for s in idx], [rhs[s] for s in idx],
                                       [g[0] for g in grids], [g[1] for g in grids], tol=tol, prec=prec,
                                       eps_inner=eps_inner, maxit_outer=maxit_outer, prune=True)
            for k, s in enumerate(idx):
                recs[s] = list(recs[s]) + list(r2[k])
    feats = np.stack([s.features(A.dim, A.grid, A.beta) for s, A in zip(systems, metas)])
    for s in systems:
        s.close()
    return recs, feats


def dataset(recs, feats):
    """(X, Y) for the systems with at least one converged trial."""
    X, Y = [], []
    for r, f in zip(recs, feats):
        t = label(r)
        if t is None:
            continue
        X.append(f)
        Y.append([math.log10(r[t]["alpha"]) - log_alpha_ref(f), r[t]["omega"]])
    return np.asarray(X, np.float32), np.asarray(Y, np.float32)


def fit(X, Y, epochs=None, lr=3e-3, seed=0, candidates=(100, 200, 400, 800, 1600, 3200), holdout=0.25):
    """Train the predictor on the device.

    With epochs=None the epoch count is chosen on a held-out split (a seeded
    quarter of the systems): each candidate count trains a fresh network on
    the rest, the one with the lowest held-out loss wins, and the final
    network is trained on everything with that count.  Returns (predictor,
    per-epoch training losses) and records the choice in `fit.last`."""
    X = np.asarray(X, np.float32)
    Y = np.asarray(Y, np.float32)
    val = None
    if epochs is None:
        rng = np.random.default_rng(seed + 7)
        idx = rng.permutation(len(X))
        k = max(1, int(holdout * len(X)))
        va, tr = idx[:k], idx[k:]
        val = {}
        for e in candidates:
            p = gadi.Predictor(seed=seed)
            p.train(X[tr], Y[tr], epochs=e, lr=lr)
            d = p.forward(X[va]) - Y[va]
            val[e] = float(np.mean(d * d))
            p.close()
        epochs = min(val, key=val.get)
    p = gadi.Predictor(seed=seed)
    losses = p.train(X, Y, epochs=epochs, lr=lr)
    fit.last = {"epochs": int(epochs), "holdout_loss": val}
    return p, losses


fit.last = {}


def save(p, path=WEIGHTS, **meta):
    mu, sd = p.norm()
    lo, hi = p.bounds()
    np.savez(path, weights=p.weights(), mu=mu, sd=sd, lo=lo, hi=hi, **meta)


def load(path=WEIGHTS):
    d = np.load(path)
    p = gadi.Predictor()
    p.set_weights(d["weights"])
    p.set_norm(d["mu"], d["sd"])
    if "lo" in d:
        p.set_bounds(d["lo"], d["hi"])
    return p


def predict(p, system, A):
    f = system.features(A.dim, A.grid, A.beta)
    return p.predict(f)


def _log_rate(hist):
    """Fitted log contraction per sweep (least squares on log RES) over the last
    third of a run's history (the early sweeps contract fast modes and overstate
    the rate), or None when the run is too short or not contracting."""
    h = np.asarray(hist, dtype=np.float64)
    h = h[np.isfinite(h) & (h > 0)]
    if len(h) < 6:
        return None
    k0 = (2 * len(h)) // 3
    slope = float(np.polyfit(np.arange(len(h))[k0:], np.log(h[k0:]), 1)[0])
    return slope if slope < 0 else None


def _projected_sweeps(hist, tol):
    """Sweeps still needed to reach RES <= tol at the fitted contraction rate."""
    slope = _log_rate(hist)
    h = np.asarray(hist, dtype=np.float64)
    if slope is None or not len(h) or not (h[-1] > 0):
        return math.inf
    return max(0.0, (math.log(tol) - math.log(h[-1])) / slope)


def default_work(system, b, tol=1e-10, **kw):
    """Work (phases) of a default-parameter solve to `tol` from x = 0 on this
    system -- the judge of a prediction -- measured by one full solve and cached
    on the handle per precision, inner tolerance and tol.  Returns (work, info
    of that solve, or None when the cached value was used); work is infinite if
    the default does not converge."""
    cache = system.__dict__.setdefault("_default_work", {})
    key = (kw.get("prec", "fp16"), kw.get("eps_inner"), float(tol))
    if key in cache:
        return cache[key], None
    _, info = system.solve(b, DEFAULT[0], DEFAULT[1], tol=tol, **kw)
    cache[key] = work(info) if info["status"] == gadi.OK else math.inf
    return cache[key], info


def _remember_default_work(system, tol, info, **kw):
    if info["status"] == gadi.OK:
        cache = system.__dict__.setdefault("_default_work", {})
        cache[(kw.get("prec", "fp16"), kw.get("eps_inner"), float(tol))] = work(info)


def solve_auto(system, A, b, predictor, tol=1e-10, probe=32, judge=None, **kw):
    """Solve with the predicted (alpha, omega); the default (0.5, 0.5) is the
    fallback and the judge.

    The judge is the work (phases of the solve kernel) a default solve to `tol`
    needs on this system: `judge` if given as a number, else the handle's cached
    value (from `default_work`, or from an earlier default solve from x = 0 in
    this function), else, with judge='measure', one default solve run first
    (its device time is reported in info['guard_seconds']).  The prediction
    runs `probe` sweeps; if that run fails (half-precision overflow,
    divergence, breakdown), the default solves from x = 0.  Otherwise the
    prediction continues from its iterate, but may spend at most the judge's
    work in total: a prediction that has not converged by then needs more work
    than the default and is rejected -- the default continues from its iterate.
    Without a judge the prediction continues unless its fitted contraction rate
    cannot reach `tol` within the sweep limit.  Returns (x, info, used) with
    used in {'mlp', 'default'}; info sums sweeps, inner steps and device seconds
    over the launches of the solve, info['fell_back'] = 1 when the default was
    used, and info['guard'] records the judge and the budget."""
    a, w = predict(predictor, system, A)
    maxit = kw.pop("maxit_outer", 20000)
    probe = min(probe, maxit)
    total = {"outer_sweeps": 0, "inner_H": 0, "inner_S": 0, "seconds": 0.0, "launches": 0}
    guard = {}
    guard_s = 0.0

    def add(info):
        info["launches"] = 1
        for k in total:
            total[k] += info[k]

    def finish(info, used, res_k=1.0):
        info.update(total)
        info["relres"] = info["relres"] * res_k
        info["fell_back"] = int(used == "default")
        info["guard_seconds"] = guard_s
        info["guard"] = guard
        return info

    if judge is None or judge == "measure":
        cache = system.__dict__.get("_default_work", {})
        key = (kw.get("prec", "fp16"), kw.get("eps_inner"), float(tol))
        if key in cache:
            judge = cache[key]
        elif judge == "measure":
            judge, dinfo = default_work(system, b, tol=tol, maxit_outer=maxit, **kw)
            guard_s += dinfo["seconds"]
        else:
            judge = None
    guard["judge_work"] = judge

    x, info = system.solve(b, a, w, tol=tol, maxit_outer=probe, history=True, **kw)
    add(info)
    if info["status"] == gadi.OK:
        return x, finish(info, "mlp"), "mlp"
    hist = system.history if system.history is not None else np.zeros(0)
    res_k = float(hist[-1]) if len(hist) else 1.0
    warm = info["status"] == gadi.EMAXIT and np.all(np.isfinite(hist)) and 0.0 < res_k < 1.0
    if warm:
        spent = work(info)
        per_sweep = spent / max(1, info["outer_sweeps"])
        if judge is not None:
            budget = int(max(0.0, judge - spent) // per_sweep) if math.isfinite(judge) else maxit - probe
            guard["budget_sweeps"] = budget
        else:
            budget = maxit - probe if _projected_sweeps(hist, tol) <= maxit - probe else 0
            guard["projected_sweeps"] = _projected_sweeps(hist, tol)
        budget = min(budget, maxit - probe)
        if budget > 0:
            x, info = system.solve(b, a, w, tol=tol / res_k, x0=x, maxit_outer=budget, **kw)
            add(info)
            if info["status"] == gadi.OK:
                return x, finish(info, "mlp", res_k), "mlp"
            if info["status"] == gadi.EMAXIT and np.all(np.isfinite(info["relres"])):
                res_k *= info["relres"]
            else:
                warm = False
    if warm:
        # over budget: the default continues from the prediction's iterate (a valid GADI start)
        x, info = system.solve(b, DEFAULT[0], DEFAULT[1], tol=tol / res_k, x0=x,
                               maxit_outer=max(1, maxit - total["outer_sweeps"]), **kw)
        add(info)
        return x, finish(info, "default", res_k), "default"
    x, info = system.solve(b, DEFAULT[0], DEFAULT[1], tol=tol, maxit_outer=maxit, **kw)
    add(info)
    _remember_default_work(system, tol, info, **kw)
    return x, finish(info, "default"), "default"
