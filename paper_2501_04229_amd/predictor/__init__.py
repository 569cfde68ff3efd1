"""(alpha, omega) prediction for GADI-IR.

The paper predicts the splitting parameter from small systems of the same
structure (Section 3.3: a training set of near-optimal parameters found on
small systems, then a regression used on large ones).  Here the regression is
the 8 -> 64 -> 64 -> 2 MLP of libgadi, trained on the device, and the training
set comes from the batched (alpha, omega) sweep of libgadi on small
convection-diffusion systems.

Label of a system: the trial with the least solver work among the trials that
reached the tolerance, where work = inner_H + 2 inner_S + 3 sweeps counts
operator products (a CG step applies alpha I + H once, a CGNE step applies S
twice, each sweep adds the residual, the first CG product and the update).
Ties go to fewer outer sweeps, then to the larger alpha.  Targets are
(log10 alpha, omega).

The default parameters (0.5, 0.5) are both the fallback and the judge:
`solve_auto` runs the predicted parameters with a work budget equal to what
the default needs (when known) and falls back to the default if the
prediction fails or runs out of budget.
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
    """Operator products of a solve record."""
    return float(rec["inner_H"] + 2 * rec["inner_S"] + 3 * rec["outer_sweeps"])


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
        Y.append([math.log10(r[t]["alpha"]), r[t]["omega"]])
    return np.asarray(X, np.float32), np.asarray(Y, np.float32)


def train(X, Y, epochs=3000, lr=3e-3, seed=0):
    p = gadi.Predictor(seed=seed)
    losses = p.train(X, Y, epochs=epochs, lr=lr)
    return p, losses


def save(p, path=WEIGHTS, **meta):
    mu, sd = p.norm()
    np.savez(path, weights=p.weights(), mu=mu, sd=sd, **meta)


def load(path=WEIGHTS):
    d = np.load(path)
    p = gadi.Predictor()
    p.set_weights(d["weights"])
    p.set_norm(d["mu"], d["sd"])
    return p


def predict(p, system, A):
    f = system.features(A.dim, A.grid, A.beta)
    return p.predict(f)


def solve_auto(system, A, b, predictor, default_work=None, **kw):
    """Solve with predicted (alpha, omega); fall back to the default parameters
    if the prediction fails or needs more work than the default (when the
    default's work is known).  Returns (x, info, used) with used in
    {'mlp', 'default'} and info['fell_back'] set accordingly."""
    a, w = predict(predictor, system, A)
    x, info = system.solve(b, a, w, **kw)
    if info["status"] == gadi.OK and (default_work is None or work(info) <= default_work):
        info["fell_back"] = 0
        return x, info, "mlp"
    x2, info2 = system.solve(b, DEFAULT[0], DEFAULT[1], **kw)
    info2["fell_back"] = 1
    info2["seconds"] += info["seconds"]
    return x2, info2, "default"
