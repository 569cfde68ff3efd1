"""Generate the (alpha, omega) sweep table on the GPU and train the predictor.

    python -m paper_2501_04229_amd.predictor.train [--systems 256] [--epochs 3000]

Training systems: gadi_inputs.train_family (small 2-D and 3-D
convection-diffusion systems, beta ~ logU(1, 500) per axis), b = A x* with
x* ~ U(-1, 1).  Every system is swept over the 16-trial grid by one batched
launch in half precision (tol 1e-10, sweep cap 5000); labels and training are
described in the package docstring.  Writes mlp_weights.npz (weights,
standardisation) and sweep_table.npz (the per-trial records) next to this file.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import gadi_inputs as gi  # noqa: E402
from paper_2501_04229_amd import predictor as pr  # noqa: E402

TABLE = os.path.join(pr.HERE, "sweep_table.npz")


def build_family(count):
    metas, rhs = [], []
    for i, (n, dim, beta) in enumerate(gi.train_family(count)):
        A = gi.convdiff(n, dim, beta)
        _, b = gi.rhs_for(A, "uniform", 1000 + i)
        metas.append(A)
        rhs.append(b)
    return metas, rhs


def features_of(metas):
    """Predictor features of each system, computed by libgadi on the device."""
    import paper_2501_04229_amd as gadi
    out = []
    for A in metas:
        g = gadi.System(A)
        out.append(g.features(A.dim, A.grid, A.beta))
        g.close()
    return np.stack(out)


def load_table(path):
    """Records (list of per-trial dicts per system) and features from a sweep table."""
    d = np.load(path)
    keys = ["status", "outer_sweeps", "inner_H", "inner_S", "relres", "seconds", "alpha", "omega"]
    recs = []
    for i in range(d["status"].shape[0]):
        row = []
        for t in range(d["status"].shape[1]):
            if np.isnan(d["status"][i, t]):
                continue
            row.append({k: (int(d[k][i, t]) if k in ("status", "outer_sweeps", "inner_H", "inner_S")
                            else float(d[k][i, t])) for k in keys})
        recs.append(row)
    return recs, d["features"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--systems", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=None,
                    help="fixed epoch count (default: chosen on a held-out quarter)")
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--maxit", type=int, default=5000)
    ap.add_argument("--out", default=pr.WEIGHTS)
    ap.add_argument("--table", default=TABLE)
    ap.add_argument("--from-table", action="store_true",
                    help="train from an existing sweep table instead of sweeping again")
    ap.add_argument("--refeature", action="store_true",
                    help="with --from-table: recompute the features of the table's systems on the device "
                         "(after a change of the feature definition) and rewrite the table")
    args = ap.parse_args()
    t0 = time.time()
    if args.from_table:
        recs, feats = load_table(args.table)
        if args.refeature:
            metas, _ = build_family(len(recs))
            feats = features_of(metas)
        t1 = t2 = time.time()
    else:
        metas, rhs = build_family(args.systems)
        t1 = time.time()
        recs, feats = pr.sweep_table(metas, rhs, maxit_outer=args.maxit)
        t2 = time.time()
    X, Y = pr.dataset(recs, feats)
    p, losses = pr.fit(X, Y, epochs=args.epochs, lr=args.lr)
    t3 = time.time()
    keys = ["status", "outer_sweeps", "inner_H", "inner_S", "relres", "seconds", "alpha", "omega"]
    width = max(len(row) for row in recs)
    table = {k: np.array([[row[t][k] if t < len(row) else np.nan for t in range(width)] for row in recs])
             for k in keys}
    if not args.from_table or args.refeature:
        np.savez(args.table, features=feats, **table)
    pr.save(p, args.out, train_loss=losses, epochs=pr.fit.last["epochs"])
    conv = int(np.nansum(table["status"] == 0))
    lab = [pr.label(r) for r in recs]
    hist = {}
    for row, t in zip(recs, lab):
        if t is not None:
            key = f"{row[t]['alpha']:.2g},{row[t]['omega']:.2g}"
            hist[key] = hist.get(key, 0) + 1
    print(json.dumps({"systems": len(recs), "trials": len(recs) * 16, "converged_trials": conv,
                      "labelled_systems": int(len(X)), "label_histogram": hist,
                      "sweep_seconds": t2 - t1, "gen_seconds": t1 - t0, "train_seconds": t3 - t2,
                      "loss_first": float(losses[0]), "loss_last": float(losses[-1]),
                      "epochs": pr.fit.last["epochs"], "holdout_loss": pr.fit.last["holdout_loss"]}), flush=True)


if __name__ == "__main__":
    main()
