"""Learned (alpha, omega) against the default on fresh 3-D systems.

    python -m paper_2501_04229_amd.predictor.evaluate [--count 40] [--nmin 96] [--nmax 192]

Test systems: gadi_inputs.test_family (3-D convection-diffusion, n ~ U{96..192},
beta ~ logU(1, 500) on all axes), b = A x* with x* ~ U(-1, 1) seeded per
system.  Each system is solved with half-precision GADI-IR to RES <= 1e-10
twice: with the default (0.5, 0.5) and with the predictor's (alpha, omega).
Reported per system and as geometric means: outer sweeps, work (phases of the
solve kernel) and device time of the raw prediction, and the device time of
`solve_auto` (the prediction guarded by the default: the default replaces it
only when a short first run fails or stalls).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import gadi_inputs as gi  # noqa: E402
import paper_2501_04229_amd as gadi  # noqa: E402
from paper_2501_04229_amd import predictor as pr  # noqa: E402


def gmean(v):
    v = [x for x in v if x > 0]
    return float(math.exp(sum(math.log(x) for x in v) / len(v))) if v else float("nan")


def evaluate(predictor, count=40, nmin=96, nmax=192, tol=1e-10, maxit_outer=20000, log=None):
    rows = []
    for (n, dim, beta, seed) in gi.test_family(count, nmin=nmin, nmax=nmax):
        A = gi.convdiff(n, dim, beta)
        xs, b = gi.rhs_for(A, "uniform", seed)
        g = gadi.System(A)
        a, w = pr.predict(predictor, g, A)
        xd, idf = g.solve(b, pr.DEFAULT[0], pr.DEFAULT[1], tol=tol, maxit_outer=maxit_outer)
        xm, iml = g.solve(b, a, w, tol=tol, maxit_outer=maxit_outer)
        xa, iau, used = pr.solve_auto(g, A, b, predictor, tol=tol, maxit_outer=maxit_outer, judge=pr.work(idf))
        ok_m = used == "mlp"
        fb_seconds = iau["seconds"]
        row = {"n": n, "beta": beta, "alpha": a, "omega": w,
               "default": {k: idf[k] for k in ("status", "outer_sweeps", "inner_H", "inner_S", "seconds")},
               "mlp": {k: iml[k] for k in ("status", "outer_sweeps", "inner_H", "inner_S", "seconds")},
               "default_work": pr.work(idf), "mlp_work": pr.work(iml), "fallback": not ok_m,
               "with_fallback_seconds": fb_seconds,
               "auto": {k: iau[k] for k in ("status", "outer_sweeps", "inner_H", "inner_S", "seconds", "relres")},
               "rel_err_auto": float(np.linalg.norm(xa - xs) / np.linalg.norm(xs)),
               "rel_err_mlp": float(np.linalg.norm(xm - xs) / np.linalg.norm(xs)),
               "rel_err_default": float(np.linalg.norm(xd - xs) / np.linalg.norm(xs))}
        rows.append(row)
        if log:
            print(f"# n={n} beta={beta:.3g} pred=({a:.3g},{w:.3g}) default {idf['outer_sweeps']} sweeps "
                  f"{idf['seconds']:.3f}s | mlp {iml['status_str']} {iml['outer_sweeps']} sweeps "
                  f"{iml['seconds']:.3f}s | auto {used} {iau['seconds']:.3f}s", file=log, flush=True)
        g.close()
    conv = [r for r in rows if r["mlp"]["status"] == gadi.OK and r["default"]["status"] == gadi.OK]
    summary = {
        "systems": len(rows),
        "both_converged": len(conv),
        "gmean_sweeps_default": gmean([r["default"]["outer_sweeps"] for r in conv]),
        "gmean_sweeps_mlp": gmean([r["mlp"]["outer_sweeps"] for r in conv]),
        "gmean_work_default": gmean([r["default_work"] for r in conv]),
        "gmean_work_mlp": gmean([r["mlp_work"] for r in conv]),
        "gmean_seconds_default": gmean([r["default"]["seconds"] for r in rows]),
        "gmean_seconds_mlp_raw": gmean([r["mlp"]["seconds"] for r in rows]),
        "gmean_seconds_mlp_with_fallback": gmean([r["with_fallback_seconds"] for r in rows]),
        "fallbacks": sum(r["fallback"] for r in rows),
        "auto_failures": sum(r["auto"]["status"] != gadi.OK for r in rows),
        "mlp_failures": sum(r["mlp"]["status"] != gadi.OK for r in rows),
    }
    summary["speedup_time_with_fallback"] = summary["gmean_seconds_default"] / summary["gmean_seconds_mlp_with_fallback"]
    summary["speedup_time_raw"] = summary["gmean_seconds_default"] / summary["gmean_seconds_mlp_raw"]
    return summary, rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=40)
    ap.add_argument("--nmin", type=int, default=96)
    ap.add_argument("--nmax", type=int, default=192)
    ap.add_argument("--weights", default=pr.WEIGHTS)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    p = pr.load(args.weights)
    t0 = time.time()
    summary, rows = evaluate(p, args.count, args.nmin, args.nmax, log=sys.stderr)
    summary["wall_seconds"] = time.time() - t0
    if args.out:
        with open(args.out, "w") as f:
            json.dump({"summary": summary, "rows": rows}, f, indent=1)
    print(json.dumps(summary), flush=True)


if __name__ == "__main__":
    main()
