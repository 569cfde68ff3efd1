"""Batched (alpha, omega) sweep throughput (the training-set generation of Section 3.3).

    python -m paper_2501_04229_amd.experiments.batched_study [--count 64] [--sequential 4]

The batched family (64 uneven 2-D convection-diffusion systems, n ~ U{128..1024},
beta ~ logU(1, 1000), seed 2, b = A 1) swept over the 16 (alpha, omega) trials
(4 log-spaced alphas in [1e-3, 10] x omega in {0, 0.5, 1, 1.5}) in one
persistent launch, FP16-IR to RES 1e-10, at most 5000 sweeps per trial.
Reported: wall time of the launch, trials per second, sweeps per second,
converged / censored trials; then the same trials of the `sequential`
smallest systems solved one by one with gadi_ir_solve for the speed-up of batching
(sweep counts must agree within max(2, 2%)), with and without the pruning of
dominated trials.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import gadi_inputs as gi  # noqa: E402
import paper_2501_04229_amd as gadi  # noqa: E402
from paper_2501_04229_amd import predictor as pr  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=64)
    ap.add_argument("--sequential", type=int, default=4)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("the batched study runs on the GPU")
    fam = gi.batched_family(a.count)
    systems, bs = [], []
    for n, dim, beta in fam:
        A = gi.convdiff(n, dim, beta)
        _, b = gi.rhs_for(A, "ones")
        systems.append(gadi.System(A))
        bs.append(b)
    rows = sum(s.n for s in systems)
    al, om = pr.trial_grid()
    res = {"systems": len(systems), "rows": rows, "trials_per_system": len(al)}
    full = None
    for prune in (True, False):
        gadi.solve_batched(systems[:2], bs[:2], al, om, tol=1e-10, maxit_outer=50, prune=prune)  # tune, warm up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        recs, _ = gadi.solve_batched(systems, bs, al, om, tol=1e-10, maxit_outer=5000, prune=prune)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        flat = [r for rs in recs for r in rs]
        ok = sum(r["status"] == gadi.OK for r in flat)
        sweeps = sum(r["outer_sweeps"] for r in flat)
        key = "pruned" if prune else "full"
        res[key] = {"seconds": dt, "trials": len(flat), "converged": ok, "sweeps": sweeps,
                    "trials_per_s": len(flat) / dt, "sweeps_per_s": sweeps / dt}
        print(f"[batched {key}] {len(flat)} trials over {len(systems)} systems ({rows} rows): {dt:.3f} s, "
              f"{len(flat) / dt:.1f} trials/s, {sweeps / dt:.0f} sweeps/s, {ok} converged", flush=True)
        if not prune:
            full = recs
    k = min(a.sequential, len(systems))
    smallest = sorted(range(len(systems)), key=lambda i: systems[i].n)[:k]
    t0 = time.perf_counter()
    agree, seq_sweeps = 0, 0
    for s in smallest:
        for t in range(len(al)):
            _, info = systems[s].solve(bs[s], al[t], om[t], tol=1e-10, maxit_outer=5000)
            seq_sweeps += info["outer_sweeps"]
            rb = full[s][t]
            if info["status"] == rb["status"] and abs(info["outer_sweeps"] - rb["outer_sweeps"]) <= max(
                    2, 0.02 * info["outer_sweeps"]):
                agree += 1
    dt_seq = time.perf_counter() - t0
    res["sequential"] = {"systems": k, "seconds": dt_seq, "sweeps": seq_sweeps, "records_agree": agree,
                         "trials": k * len(al), "rows": sum(systems[i].n for i in smallest)}
    print(f"[sequential] the {k} smallest systems, {k * len(al)} trials one by one: {dt_seq:.3f} s; "
          f"{agree}/{k * len(al)} records agree with the batched launch", flush=True)
    for s in systems:
        s.close()
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
    print(json.dumps({"batched_study": True}))


if __name__ == "__main__":
    main()
