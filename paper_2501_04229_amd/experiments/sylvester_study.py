"""GADI-AB on the continuous Sylvester equation of Section 4.3.

    python -m paper_2501_04229_amd.experiments.sylvester_study [--n 64] [--budget 100000] [--out FILE]

Part 1 (the section's table): for r in {0.01, 0.1, 1} and alpha in
{0.01, 0.02, 10}, half-precision inner solves (and double ones beside them)
run with an unreachable tolerance until RES stops improving, fails, or a sweep
budget is spent; reported are the smallest relative residual
RES = ||C - A X - X B||_F / ||C||_F reached, the sweep where it was reached and
the status.

Part 2 (the section's figure): the same smallest RES over a log grid of alpha
in [0.01, 10] for each r, half-precision inner solves.

Part 3: device time per sweep at n = 1024 and 4096 (r = 0.1, alpha = 0.5) for
the three inner precisions, with the sweep's algorithmic HBM bytes per element
(double X and C, inner-type work arrays) and the rate they imply.
--copy-calibration ends the run with one elementwise copy of known size, so that
hardware byte counters taken over the run can be scaled to bytes.

A = B = M + 2 r N + 100/(n+1)^2 I, M = Tridiag(-1, 2, -1), N = Tridiag(0.5, 0,
-0.5); the right-hand side is C = A 1 + 1 B, so X* = 1 (all ones).  The section
prints neither n, omega nor the tolerance: n is a parameter, omega = 0.5.
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

RS = (0.01, 0.1, 1.0)
ALPHAS = (0.01, 0.02, 10.0)
# algorithmic bytes per matrix element per sweep: residual (X, C read, R
# written), column solves (R read, z^ written), row solves (z^ read, y^
# written), update (y^ read, X read and written)
BYTES = {"fp64": 8 + 8 + 8 + 8 + 8 + 8 + 8 + 8 + 8 + 8, "fp32": 8 + 8 + 4 + 4 + 4 + 4 + 4 + 4 + 8 + 8,
         "fp16": 8 + 8 + 4 + 4 + 4 + 4 + 4 + 4 + 8 + 8}


def system(n, r, device):
    import torch
    A = gi.paper_tridiag(n, r)
    Xs, C = gi.sylvester_rhs(A, A, "ones")
    Cd = torch.from_numpy(C).to(device)
    return gadi.Sylvester(A, A), Cd


def attainable(g, C, al, omega, prec, chunk, budget, tol=1e-15):
    """Smallest RES: warm-started launches of `chunk` sweeps until a launch
    fails, RES stops improving by 10% over a launch, RES <= tol, or `budget`
    sweeps have been spent.  RES stays relative to ||C|| across launches."""
    x, scale, best, at, done, status, secs, limited = None, 1.0, math.inf, 0, 0, "stalled", 0.0, False
    while True:
        if done >= budget:
            limited = True
            status = "budget"
            break
        x, info = g.solve(C, al, omega, tol=tol / scale, prec=prec, maxit_outer=min(chunk, budget - done),
                          history=True, x0=x)
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
        if info["status"] == gadi.OK:
            status = "ok"
            break
        if not improved:
            break
        scale = float(h[-1])
    return {"res": best if best < math.inf else None, "at": at, "sweeps": done, "status": status,
            "budget_limited": limited, "seconds": secs}


def part1(n, omega, chunk, budget, device):
    rows = []
    for r in RS:
        g, C = system(n, r, device)
        for al in ALPHAS:
            for prec in ("fp16", "fp64"):
                t = attainable(g, C, al, omega, prec, chunk, budget)
                t.update({"r": r, "alpha": al, "prec": prec})
                rows.append(t)
                print(f"[table] n={n} r={r} alpha={al} {prec}: RES {t['res']:.3e} at sweep {t['at']} "
                      f"({t['status']}, {t['sweeps']} sweeps, {t['seconds']:.2f} s)", flush=True)
        g.close()
    return rows


def part2(n, omega, chunk, budget, device, points):
    rows = []
    grid = np.logspace(-2, 1, points)
    for r in RS:
        g, C = system(n, r, device)
        for al in grid:
            t = attainable(g, C, float(al), omega, "fp16", chunk, budget)
            t.update({"r": r, "alpha": float(al), "prec": "fp16"})
            rows.append(t)
            print(f"[alpha] n={n} r={r} alpha={al:.4g}: RES {t['res']:.3e} at sweep {t['at']} ({t['status']})",
                  flush=True)
        g.close()
    return rows


def part3(sizes, device, sweeps):
    rows = []
    for n in sizes:
        g, C = system(n, 0.1, device)
        for prec in ("fp64", "fp32", "fp16"):
            g.solve(C, 0.5, 0.5, tol=0.0, prec=prec, maxit_outer=3)
            _, info = g.solve(C, 0.5, 0.5, tol=0.0, prec=prec, maxit_outer=sweeps)
            us = info["seconds"] / info["outer_sweeps"] * 1e6
            gbs = BYTES[prec] * n * n / (us * 1e-6) / 1e9
            rows.append({"n": n, "prec": prec, "us_per_sweep": us, "bytes_per_element": BYTES[prec], "GB_s": gbs})
            print(f"[time] n={n} {prec}: {us:.1f} us/sweep, {BYTES[prec]} B/element, {gbs:.0f} GB/s", flush=True)
        g.close()
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--omega", type=float, default=0.5)
    ap.add_argument("--chunk", type=int, default=2000)
    ap.add_argument("--budget", type=int, default=100000)
    ap.add_argument("--points", type=int, default=13)
    ap.add_argument("--time-sweeps", type=int, default=500)
    ap.add_argument("--parts", default="123")
    ap.add_argument("--out", default=None)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with one elementwise copy of 2^26 floats (reads and writes 256 MiB) "
                         "to calibrate hardware byte counters")
    a = ap.parse_args()
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("the Sylvester study runs on the GPU")
    dev = torch.device("cuda:0")
    t0 = time.time()
    res = {"n": a.n, "omega": a.omega, "budget": a.budget}
    if "1" in a.parts:
        res["table"] = part1(a.n, a.omega, a.chunk, a.budget, dev)
    if "2" in a.parts:
        res["alpha_grid"] = part2(a.n, a.omega, a.chunk, a.budget, dev, a.points)
    if "3" in a.parts:
        res["timing"] = part3((1024, 4096), dev, a.time_sweeps)
    res["wall_seconds"] = time.time() - t0
    if a.copy_calibration:
        xc = torch.ones(1 << 26, device=dev, dtype=torch.float32)
        yc = torch.empty_like(xc)
        torch.mul(xc, 1.0, out=yc)
        torch.cuda.synchronize()
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
    print(json.dumps({"wall_seconds": res["wall_seconds"]}))


if __name__ == "__main__":
    main()
