"""Batched (alpha, omega) sweep throughput (the training-set generation of Section 3.3).

    python -m paper_2501_04229_amd.experiments.batched_study [--count 64] [--group 16] [--sequential 4]

The batched family (uneven 2-D convection-diffusion systems, n ~ U{128..1024},
beta ~ logU(1, 1000), seed 2, b = A 1) swept over the 16 (alpha, omega) trials
(4 log-spaced alphas in [1e-3, 10] x omega in {0, 0.5, 1, 1.5}), FP16-IR to
RES 1e-10, at most 5000 sweeps per trial, with dominated trials pruned (a trial
stops once its work exceeds that of a converged trial of its system).  The
family runs in launches of `group` systems (default: all of them in one
launch), each reported when it ends: wall time, trials per second, sweeps per
second, converged and pruned trials, and the matrix bytes a trial reads per
product with and without the pack's shared matrix loads.  Then the
`sequential` smallest systems:
one unpruned batched launch against the same trials solved one by one with
gadi_ir_solve in the same inner form (records must agree: status, sweeps within
max(2, 2%)).
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


def build(fam):
    systems, bs = [], []
    for n, dim, beta in fam:
        A = gi.convdiff(n, dim, beta)
        _, b = gi.rhs_for(A, "ones")
        systems.append(gadi.System(A))
        bs.append(b)
    return systems, bs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=64)
    ap.add_argument("--group", type=int, default=0, help="systems per launch (0: all in one launch)")
    ap.add_argument("--sequential", type=int, default=4)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("the batched study runs on the GPU")
    fam = gi.batched_family(a.count)
    al, om = pr.trial_grid()
    group = a.group or len(fam)
    os.environ["GADI_PROGRESS"] = "1"
    res = {"systems": len(fam), "trials_per_system": len(al), "groups": []}
    tot_t, tot_trials, tot_sweeps, tot_ok, tot_rows = 0.0, 0, 0, 0, 0
    for g0 in range(0, len(fam), group):
        t0 = time.perf_counter()
        systems, bs = build(fam[g0:g0 + group])
        t_setup = time.perf_counter() - t0
        rows = sum(s.n for s in systems)
        gadi.solve_batched(systems[:1], bs[:1], al, om, tol=1e-10, maxit_outer=20, prune=True)  # tuner, warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        recs, _ = gadi.solve_batched(systems, bs, al, om, tol=1e-10, maxit_outer=5000, prune=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        flat = [r for rs in recs for r in rs]
        ok = sum(r["status"] == gadi.OK for r in flat)
        sweeps = sum(r["outer_sweeps"] for r in flat)
        # fp16 operator bytes per row of one product (values of the 2-D stencil's H with its
        # diagonal, or of S): read once per pack of up to 4 trials instead of once per trial
        lay = [s_.layout() for s_ in systems]
        mat = sum(2.0 * (L["nnz_off"] + L["n"]) for L in lay) / max(1, sum(L["n"] for L in lay))
        res["groups"].append({"first": g0, "systems": len(systems), "rows": rows, "seconds": dt, "setup_s": t_setup,
                              "trials": len(flat), "converged": ok, "sweeps": sweeps,
                              "maxit": sum(r["status"] == gadi.EMAXIT for r in flat),
                              "pruned": sum(r["status"] == gadi.EPRUNED for r in flat),
                              "matrix_bytes_per_row_product_unshared": mat,
                              "matrix_bytes_per_row_product_per_trial": mat / 4.0,
                              "sweeps_per_s": sweeps / dt, "trials_per_s": len(flat) / dt,
                              "launch_seconds": flat[0]["barrier_seconds"]})
        tot_t += dt
        tot_trials += len(flat)
        tot_sweeps += sweeps
        tot_ok += ok
        tot_rows += rows
        print(f"[batched] systems {g0}..{g0 + len(systems) - 1} ({rows} rows): {len(flat)} trials in {dt:.3f} s, "
              f"{len(flat) / dt:.1f} trials/s, {sweeps / dt:.0f} sweeps/s, {ok} converged (setup {t_setup:.1f} s)",
              flush=True)
        for s in systems:
            s.close()
    res["total"] = {"seconds": tot_t, "trials": tot_trials, "converged": tot_ok, "sweeps": tot_sweeps,
                    "rows": tot_rows, "trials_per_s": tot_trials / tot_t, "sweeps_per_s": tot_sweeps / tot_t}
    print(f"[batched total] {tot_trials} trials, {tot_rows} rows: {tot_t:.3f} s, {tot_trials / tot_t:.1f} trials/s, "
          f"{tot_ok} converged", flush=True)

    small = sorted(fam, key=lambda f: f[0])[:a.sequential]
    systems, bs = build(small)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs, _ = gadi.solve_batched(systems, bs, al, om, tol=1e-10, maxit_outer=5000, prune=False)
    torch.cuda.synchronize()
    dt_b = time.perf_counter() - t0
    print(f"[batched unpruned] the {len(systems)} smallest systems: {dt_b:.3f} s", flush=True)
    # the single solves run the batched kernel's inner form (Chronopoulos-Gear), so that the
    # records compare the same iterations (the other forms differ in rounding and, at the smallest
    # alpha, in where half precision overflows)
    os.environ["GADI_SOLVE_FORM"] = "1"
    t0 = time.perf_counter()
    agree = 0
    status_agree = 0
    for s in range(len(systems)):
        for t in range(len(al)):
            _, info = systems[s].solve(bs[s], al[t], om[t], tol=1e-10, maxit_outer=5000)
            rb = recs[s][t]
            status_agree += int(info["status"] == rb["status"])
            if info["status"] == rb["status"] and abs(info["outer_sweeps"] - rb["outer_sweeps"]) <= max(
                    2, 0.02 * info["outer_sweeps"]):
                agree += 1
        print(f"[sequential] system {s} done", flush=True)
    dt_s = time.perf_counter() - t0
    res["sequential"] = {"systems": len(systems), "batched_seconds": dt_b, "sequential_seconds": dt_s,
                         "records_agree": agree, "status_agree": status_agree, "trials": len(systems) * len(al)}
    print(f"[sequential] {len(systems) * len(al)} trials one by one: {dt_s:.3f} s against {dt_b:.3f} s batched; "
          f"{agree}/{len(systems) * len(al)} records agree (status {status_agree}/{len(systems) * len(al)})",
          flush=True)
    for s in systems:
        s.close()
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
    print(json.dumps({"batched_study": True}))


if __name__ == "__main__":
    main()
