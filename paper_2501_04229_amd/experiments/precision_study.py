"""The precision study of Section 4.1 on a synthetic 3-D convection-diffusion system.

    python -m paper_2501_04229_amd.experiments.precision_study [--n 64] [--beta 20] [--budget 3000]

Part 1 (Table 3d): for alpha in {0.01, 0.02, 10} and the precision triples
(u_r, u, u_f) of the table, run GADI-IR with an unreachable tolerance until
RES stops improving (or a sweep budget) and report the smallest relative
residual RES reached (the table's RRES), the sweep where it was reached, and
the status ("-" in the table's sense when a run failed: half overflow,
divergence, breakdown).

Part 2 (Table "alpha-effects"): half-precision inner solves with double outer
precisions over the table's alphas: sweeps to RES <= 1e-10 and the device time.

The matrix is the table's family (h^2-scaled 3-D convection-diffusion, beta on
all axes, b = A 1); the paper prints no grid size, omega or tolerance, so these
are parameters here (omega = 0.5).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import gadi_inputs as gi  # noqa: E402
import paper_2501_04229_amd as gadi  # noqa: E402

TRIPLES = [("double", "double", "double", "fp64"), ("single", "single", "single", "s-s-s"),
           ("single", "double", "double", "fp32"), ("half", "double", "single", "h-d-s"),
           ("half", "double", "double", "fp16"), ("half", "single", "single", "h-s-s")]


def attainable(g, b, al, omega, prec, chunk, budget, seconds, tol=1e-15):
    """Smallest RES reached: warm-started launches of `chunk` sweeps until a
    launch fails, RES stops improving by 10% over a launch, RES <= tol, or
    `budget` sweeps or `seconds` of device time have been spent (then the
    result is marked budget-limited).  RES stays relative to ||b|| across
    launches (each launch reports it relative to its own start)."""
    eps = 1e-6 if prec == "fp64" else 1e-3
    x, scale, best, at, done, status, secs, limited = None, 1.0, math.inf, 0, 0, "ok", 0.0, False
    while True:
        if done >= budget or secs >= seconds:
            limited = True
            break
        x, info = g.solve(b, al, omega, tol=tol / scale, prec=prec, eps_inner=eps,
                          maxit_outer=min(chunk, budget - done), history=True, x0=x)
        secs += info["seconds"]
        h = np.asarray(g.history) * scale
        if info["status"] not in (gadi.OK, gadi.EMAXIT) or not len(h):
            status = info["status_str"]
            break
        k = int(np.argmin(h))
        improved = h[k] < 0.9 * best
        if h[k] < best:
            best, at = float(h[k]), done + k
        done += info["outer_sweeps"]
        scale = float(h[-1])
        print(f"#   {prec} alpha {al:g}: {done} sweeps, RES {best:.3g}, {secs:.1f} s", file=sys.stderr, flush=True)
        if info["status"] == gadi.OK or not improved or best <= tol:
            break
    if status == "ok" and not best < 0.5:
        status = "no progress"  # RES never fell below 1/2: the table's "-"
    return status, (best if status == "ok" else None), at, done, secs, limited


def part1(g, b, alphas, omega, chunk, budget, seconds):
    rows = []
    for al in alphas:
        for ur, u, uf, prec in TRIPLES:
            status, rres, at, done, secs, limited = attainable(g, b, al, omega, prec, chunk, budget, seconds)
            rows.append({"alpha": al, "u_r": ur, "u": u, "u_f": uf, "status": status, "rres": rres,
                         "at_sweep": at, "sweeps": done, "seconds": secs, "budget_limited": limited})
            print(f"# alpha {al:g} ({ur}, {u}, {uf}): {status} min RES {fmt(rres)} at sweep {at} of {done}"
                  f"{' (budget-limited)' if limited else ''}", file=sys.stderr, flush=True)
    return rows


def part2(g, b, alphas, omega, chunk, budget, seconds):
    rows = []
    for al in alphas:
        status, rres, at, done, secs, limited = attainable(g, b, al, omega, "fp16", chunk, budget, seconds, tol=1e-10)
        rows.append({"alpha": al, "status": status, "sweeps": done, "min_res": rres, "seconds": secs,
                     "budget_limited": limited})
        print(f"# alpha {al:g}: {status} sweeps {done} RES {fmt(rres)}", file=sys.stderr, flush=True)
    return rows


def fmt(v):
    return "-" if v is None else f"{v:.1e}"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=32)
    ap.add_argument("--beta", type=float, default=20.0)
    ap.add_argument("--omega", type=float, default=0.5)
    ap.add_argument("--budget", type=int, default=40000)
    ap.add_argument("--chunk", type=int, default=500)
    ap.add_argument("--seconds", type=float, default=15.0, help="device-time cap per configuration")
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    A = gi.convdiff(args.n, 3, args.beta)
    _, b = gi.rhs_for(A, "ones")
    g = gadi.System(A)
    t1 = part1(g, b, (0.01, 0.02, 10.0), args.omega, args.chunk, args.budget, args.seconds)
    t2 = part2(g, b, (0.01, 0.02, 0.05, 0.1, 0.5, 1.0, 5.0, 10.0, 100.0), args.omega, args.chunk, args.budget,
               args.seconds)
    out = {"n": args.n, "beta": args.beta, "omega": args.omega, "budget": args.budget, "table_3d": t1,
           "alpha_effects": t2}
    if args.out:
        with open(args.out, "w") as f:
            json.dump(out, f, indent=1)
    print(f"Table 3d reproduction: 3-D n = {args.n}, beta = {args.beta}, omega = {args.omega}, b = A 1; "
          f"RRES = smallest RES reached (launches of {args.chunk} sweeps until RES stops improving, "
          f"at most {args.budget} sweeps)")
    print("| u_r | u | u_f | alpha | RRES | at sweep | sweeps run | seconds |")
    print("|---|---|---|---|---|---|---|---|")
    for r in t1:
        lim = " (budget)" if r["budget_limited"] else ""
        print(f"| {r['u_r']} | {r['u']} | {r['u_f']} | {r['alpha']:g} | {fmt(r['rres'])}{lim} | {r['at_sweep']} | "
              f"{r['sweeps']} | {r['seconds']:.2f} |")
    print()
    print("alpha effects, (half, double, double), to RES <= 1e-10:")
    print("| alpha | status | sweeps | RES | seconds |")
    print("|---|---|---|---|---|")
    for r in t2:
        lim = " (budget)" if r["budget_limited"] else ""
        print(f"| {r['alpha']:g} | {r['status']} | {r['sweeps']}{lim} | {fmt(r['min_res'])} | {r['seconds']:.3f} |")


if __name__ == "__main__":
    main()
