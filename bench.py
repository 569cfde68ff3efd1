#!/usr/bin/env python3
"""Benchmark: time-to-1e-10 of FP16-IR GADI vs plain FP64 GADI on one MI355X.

One step = one complete GADI-IR solve (every hot-path phase: FP64 residual,
CG on alpha I + H, CGNE on alpha I + S, FP64 update, repeated to RES <= 1e-10)
of the 3-D convection-diffusion system, 128^3 grid, beta = (20, 20, 20),
b = A x* with x* ~ U(-1, 1) seed 0, inputs resident in device memory.

Prints one JSON line.  The plain FP64 GADI solve (inner CG/CGNE to 1e-6) is
timed on the same GPU for the comparison; the FP64 CPU oracle is timed on a
bounded sample of outer sweeps on the host cores (cpu_baseline leg).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-1e-10 residual & SpMV HBM GB/s: FP16-IR+MLP vs plain FP64 GADI"
HBM_PEAK_GBS = 8000.0
WEIGHTS = os.path.join(ROOT, "paper_2501_04229_amd", "predictor", "mlp_weights.npz")


def solve_bytes(prec: str, L: dict, sweeps: int, inner_h: int, inner_s: int, launches: int = 1) -> float:
    """Algorithmic HBM bytes of solve-kernel launches with the given iteration counts.

    Matrix streams follow the packed layout (L = System.layout()): one value per
    structural entry plus an int32 column for entries of explicit slices
    (diagonal-style slices store no column).  Per unit, with N rows, z_o
    off-diagonal entries, z_e of them in explicit slices, m / d / v = bytes of an
    off-diagonal value / a diagonal value / a vector entry (fp16 2/2/2, fp32 4/4/4,
    fp64 8/8/8, fp8 1/2/2: E4M3 values, half diagonal and vectors), s = inner
    accumulator bytes (4, or 8 in fp64):
      residual a1          8 (z_o + N) + 4 z_e + 22 N          (double A, x, b; scaled output)
      CG step              m z_o + d N + 4 z_e + 8 v N         (alpha I + H product, 8 vector accesses)
      CGNE step            2 (m z_o + 4 z_e + 4 v N)           (two S products)
      update a6            m z_o + 4 z_e + 16 N + 2 s N        (one S product, x read/write)
    Each launch evaluates one residual more than it applies corrections."""
    m, d, v = {"fp16": (2, 2, 2), "fp32": (4, 4, 4), "fp64": (8, 8, 8), "fp8": (1, 2, 2)}[prec]
    sb = 8 if prec == "fp64" else 4
    n, zo, ze = L["n"], L["nnz_off"], L["explicit_entries"]
    res = 8 * (zo + n) + 4 * ze + 22 * n
    cg = m * zo + d * n + 4 * ze + 8 * v * n
    cgne = 2 * (m * zo + 4 * ze + 4 * v * n)
    upd = m * zo + 4 * ze + 16 * n + 2 * sb * n
    return float((sweeps + launches) * res + sweeps * upd + inner_h * cg + inner_s * cgne)


def profiled_traffic(workload: str, prec: str):
    """HBM bytes per solve launch from the committed rocprofv3 counter summary of
    this workload (profiles/solve_kernel_<prec>_<workload>_traffic.md: FETCH_SIZE
    and WRITE_SIZE runs, copy-calibrated, over the timed launches), or None if
    there is none or the kernel sources, predictor or workload generator have
    changed since the counters were taken (source hash mismatch)."""
    path = os.path.join(ROOT, "profiles", f"solve_kernel_{prec}_{workload}_traffic.md")
    if not os.path.exists(path):
        return None, "no counter summary"
    vals = {}
    with open(path) as f:
        for line in f:
            line = line.strip().strip("`")
            for key in ("traffic_bytes_per_launch", "source_sha256"):
                if line.startswith(key + ":"):
                    vals[key] = line.split(":", 1)[1].strip()
    from paper_2501_04229_amd.rocprof_summary import source_hash
    if vals.get("source_sha256") != source_hash(ROOT) or "traffic_bytes_per_launch" not in vals:
        return None, f"{os.path.relpath(path, ROOT)} is stale (sources changed since the counters were taken)"
    return float(vals["traffic_bytes_per_launch"]), os.path.relpath(path, ROOT)


def load_predictor():
    """The trained (alpha, omega) predictor, or None if no weights are present."""
    if not os.path.exists(WEIGHTS):
        return None
    from paper_2501_04229_amd import predictor as pr
    return pr.load(WEIGHTS)


def cpu_baseline(A, b, alpha, omega, sweeps_needed, eps, budget_s=20.0, threads=0):
    """FP64 oracle (plain GADI, the same algorithm) on the host: time a bounded
    number of outer sweeps and scale per sweep to the sweeps the solve needs.
    threads > 0 sets the oracle's OpenMP threads (default: all it is given)."""
    import oracle
    if threads > 0:
        oracle.set_num_threads(threads)
    o = oracle.OracleSystem(A)
    k = 1
    t0 = time.perf_counter()
    r = o.gadi(b, alpha, omega, tol=0.0, eps_h=eps, eps_s=eps, maxit_out=k)
    t1 = time.perf_counter()
    per = (t1 - t0) / k
    k2 = max(1, min(int(budget_s / max(per, 1e-6)), 50))
    t0 = time.perf_counter()
    r = o.gadi(b, alpha, omega, tol=0.0, eps_h=eps, eps_s=eps, maxit_out=k2)
    t1 = time.perf_counter()
    per = (t1 - t0) / k2
    return {
        "value": per * sweeps_needed,
        "unit": "s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"{k2} FP64 GADI sweeps (inner CG/CGNE to {eps:g}) of the same system timed, "
                  f"{per:.3f} s/sweep, scaled to the {sweeps_needed} sweeps plain FP64 GADI needs",
        "seconds_per_sweep": per,
        "sample_sweeps": k2,
        "inner_h_per_sweep": r["inner_h"] / max(1, r["sweeps"]),
    }


def _graph_time(fn, out, reps):
    """Device seconds per call of fn, whose kernels the library enqueues on the
    current stream: reps calls are captured in one graph and replayed, so
    host-side call overhead does not count.  Every replay's output is checked
    against an eager call's (the products are deterministic)."""
    import torch
    fn()
    torch.cuda.synchronize()
    ref = out.clone()
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gr):
        for _ in range(reps):
            fn()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(3):
        out.zero_()
        torch.cuda.synchronize()
        e0.record()
        gr.replay()
        e1.record()
        torch.cuda.synchronize()
        if not torch.equal(out, ref):
            raise RuntimeError("a graph replay of the product differs from the eager call")
        best = min(best, e0.elapsed_time(e1) * 1e-3 / reps)
    return best


def spmv_gbs(g, A, alpha, reps=50):
    """Stand-alone products: fp16 (alpha I + H) x moves 2 (z_o + N) + 4 z_e + 4 N
    algorithmic bytes, fp64 A x moves 8 (z_o + N) + 4 z_e + 16 N.  Device time
    per product from a replayed graph of reps products."""
    import torch
    n = A.n
    gen = torch.Generator(device="cuda").manual_seed(5)
    x = torch.rand(n, device="cuda", dtype=torch.float16, generator=gen)
    y = torch.empty_like(x)
    dt = _graph_time(lambda: g.spmv("H16", x, y, alpha), y, reps)
    L = g.layout()
    by = 2.0 * (L["nnz_off"] + n) + 4.0 * L["explicit_entries"] + 4.0 * n
    x64 = torch.rand(n, device="cuda", dtype=torch.float64, generator=gen)
    y64 = torch.empty_like(x64)
    dt64 = _graph_time(lambda: g.spmv("A", x64, y64), y64, reps)
    by64 = 8.0 * (L["nnz_off"] + n) + 4.0 * L["explicit_entries"] + 16.0 * n
    return {"fp16_H_us": dt * 1e6, "fp16_H_GBs": by / dt / 1e9, "fp64_A_us": dt64 * 1e6,
            "fp64_A_GBs": by64 / dt64 / 1e9, "timing": "graph of %d products, best of 3 replays" % reps}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="convdiff3d_128_beta20")
    ap.add_argument("--prec", default="fp16", choices=["fp16", "fp32", "fp64", "fp8"])
    ap.add_argument("--eps-inner", type=float, default=None)
    ap.add_argument("--params", default="mlp", choices=["mlp", "default"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-spmv", action="store_true", help="skip the stand-alone product timing (graph replays)")
    ap.add_argument("--cpu-threads", type=int, default=0, help="OpenMP threads of the oracle timing (0: all)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with one elementwise copy of 2^26 floats (reads and writes 256 MiB) "
                         "to calibrate hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the solver is a single-GPU build.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import gadi_inputs as gi
    import paper_2501_04229_amd as gadi

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    t_setup = time.perf_counter()
    W = gi.workload(args.workload)
    A, b, xs = W["A"], W["b"], W["xstar"]
    g = gadi.System(A)
    setup_s = time.perf_counter() - t_setup
    z = A.nnz
    zs = A.nnz - A.n
    n = A.n
    bd = torch.from_numpy(b).cuda()
    eps = args.eps_inner
    pred = load_predictor() if args.params == "mlp" else None
    from paper_2501_04229_amd import predictor as pr
    alpha, omega, psrc = 0.5, 0.5, "default"
    if pred is not None:
        alpha, omega = pr.predict(pred, g, A)
        psrc = "mlp"

    def run(prec, al, om, e):
        """One step: with the predictor, solve_auto (prediction guarded by the default);
        without, a plain solve.  Returns (x, info, launches, used)."""
        if pred is not None and prec == args.prec:
            x, info, used = pr.solve_auto(g, A, bd, pred, tol=1e-10, prec=prec, eps_inner=e)
            return x, info, info["launches"], used
        x, info = g.solve(bd, al, om, tol=1e-10, prec=prec, eps_inner=e)
        return x, info, 1, "fixed"

    print(f"# workload {args.workload}: N={n} nnz={z} setup {setup_s:.1f}s params {psrc} "
          f"alpha={alpha:.4g} omega={omega:.4g}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        x, info, nl, used = run(args.prec, alpha, omega, eps)
        print(f"# warmup: {info['status_str']} used={used} sweeps={info['outer_sweeps']} inner_H={info['inner_H']} "
              f"inner_S={info['inner_S']} {info['seconds']:.3f}s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kernel_s = []
    infos = []
    launches = 0
    for _ in range(args.steps):
        x, info, nl, used = run(args.prec, alpha, omega, eps)
        kernel_s.append(info["seconds"])
        infos.append(info)
        launches += nl
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    step_s = (t1 - t0) / args.steps
    info = infos[-1]
    if info["status"] != gadi.OK:
        print(f"# solve did not converge: {info}", file=sys.stderr, flush=True)
    prof = g.phase_profile()
    print("# phase profile (block 0 compute s, count): " +
          ", ".join(f"{k} {v[0]:.4f}/{v[1]}" for k, v in prof.items() if v[1]), file=sys.stderr, flush=True)
    xh = x.cpu().numpy()
    rel_err_xstar = float(np.linalg.norm(xh - xs) / np.linalg.norm(xs))
    kern = float(np.mean(kernel_s))
    # every solve-kernel launch of the timed region: total algorithmic bytes / total device time
    lay = g.layout()
    tot_bytes = 0.0
    for inf in infos:
        tot_bytes += solve_bytes(args.prec, lay, inf["outer_sweeps"], inf["inner_H"], inf["inner_S"],
                                 inf.get("launches", 1))
    nbytes = tot_bytes / launches
    achieved = tot_bytes / float(np.sum(kernel_s)) / 1e9
    print(f"# {args.prec}-IR: {step_s:.3f}s/solve, kernel {kern:.3f}s, {achieved:.0f} GB/s algorithmic, "
          f"sweeps={info['outer_sweeps']} inner_H={info['inner_H']} inner_S={info['inner_S']} "
          f"relres={info['relres']:.3e} err_vs_x*={rel_err_xstar:.3e} barriers={info['barriers']} "
          f"block0 in barriers {info['barrier_seconds']:.3f}s", file=sys.stderr, flush=True)

    # the same precision with the default parameters, no predictor (reference)
    xdf, idf = g.solve(bd, 0.5, 0.5, tol=1e-10, prec=args.prec, eps_inner=eps)
    torch.cuda.synchronize()
    fp16_default = {"seconds": idf["seconds"], "status": idf["status_str"], "sweeps": idf["outer_sweeps"],
                    "inner_H": idf["inner_H"], "inner_S": idf["inner_S"], "relres": idf["relres"]}
    print(f"# {args.prec} default (0.5, 0.5): {idf['seconds']:.3f}s sweeps={idf['outer_sweeps']}",
          file=sys.stderr, flush=True)

    fp64 = None
    if not args.no_fp64:
        run("fp64", 0.5, 0.5, 1e-6)  # first call tunes the FP64 launch shape
        torch.cuda.synchronize()
        tf0 = time.perf_counter()
        x64, i64, _, _ = run("fp64", 0.5, 0.5, 1e-6)
        torch.cuda.synchronize()
        wall64 = time.perf_counter() - tf0
        x64h = x64.cpu().numpy()
        nb64 = solve_bytes("fp64", lay, i64["outer_sweeps"], i64["inner_H"], i64["inner_S"])
        fp64 = {"seconds": i64["seconds"], "wall_seconds": wall64, "status": i64["status_str"],
                "sweeps": i64["outer_sweeps"],
                "inner_H": i64["inner_H"], "inner_S": i64["inner_S"], "relres": i64["relres"],
                "rel_err_vs_xstar": float(np.linalg.norm(x64h - xs) / np.linalg.norm(xs)),
                "algorithmic_GBs": nb64 / i64["seconds"] / 1e9,
                "rel_diff_vs_fp16ir": float(np.linalg.norm(xh - x64h) / np.linalg.norm(x64h))}
        print(f"# fp64 GADI: {i64['seconds']:.3f}s sweeps={i64['outer_sweeps']} inner_H={i64['inner_H']} "
              f"inner_S={i64['inner_S']} relres={i64['relres']:.3e}", file=sys.stderr, flush=True)
        # the same plain FP64 GADI with the reduced-precision solve's inner tolerance: separates the
        # effect of the precision from that of the inner tolerance (informational)
        eps_rp = gadi.options(args.prec).eps_inner
        torch.cuda.synchronize()
        tf0 = time.perf_counter()
        _, i64e, _, _ = run("fp64", 0.5, 0.5, eps_rp)
        torch.cuda.synchronize()
        fp64["same_inner_eps"] = {"eps_inner": eps_rp, "seconds": i64e["seconds"],
                                  "wall_seconds": time.perf_counter() - tf0, "status": i64e["status_str"],
                                  "sweeps": i64e["outer_sweeps"], "inner_H": i64e["inner_H"],
                                  "inner_S": i64e["inner_S"]}
        print(f"# fp64 GADI, inner {eps_rp:g}: {i64e['seconds']:.3f}s sweeps={i64e['outer_sweeps']}",
              file=sys.stderr, flush=True)
    sp = None
    if not args.no_spmv:
        sp = spmv_gbs(g, A, alpha)
        print(f"# spmv: {sp}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu:
        sweeps_needed = fp64["sweeps"] if fp64 else info["outer_sweeps"]
        cpu = cpu_baseline(A, b, 0.5, 0.5, sweeps_needed, 1e-6, threads=args.cpu_threads)
        print(f"# cpu oracle: {cpu['seconds_per_sweep']:.3f}s/sweep on {cpu['cores']} threads -> "
              f"{cpu['value']:.1f}s", file=sys.stderr, flush=True)

    out = {
        "metric": METRIC,
        "value": step_s,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": {"fp16": "fp16 storage / fp32 arithmetic inner, f64 residual+update",
                  "fp32": "f32 inner, f64 residual+update", "fp64": "f64",
                  "fp8": "e4m3 values, fp16 vectors / fp32 arithmetic inner, f64 residual+update"}[args.prec],
        "data": "synthetic",
        "layout": lay,
        "config": {"workload": args.workload, "N": n, "nnz": z, "tol": 1e-10,
                   "eps_inner": eps if eps is not None else gadi.options(args.prec).eps_inner,
                   "alpha_predicted": alpha, "omega_predicted": omega, "params": psrc, "used": used,
                   "prec": args.prec,
                   "solve_launch_blocks_threads": list(g.solver_blocks())},
        "solve": {"status": info["status_str"], "sweeps": info["outer_sweeps"], "inner_H": info["inner_H"],
                  "inner_S": info["inner_S"], "relres": info["relres"], "rel_err_vs_xstar": rel_err_xstar,
                  "kernel_seconds": kern, "barriers": info["barriers"],
                  "barrier_seconds_block0": info["barrier_seconds"]},
        "default_params_same_prec": fp16_default,
        "fp64_gadi": fp64,
        "speedup_vs_fp64_gadi": (fp64["wall_seconds"] / step_s) if fp64 else None,
        "spmv": sp,
        "phase_profile_last_launch": {k: {"seconds": v[0], "count": v[1]} for k, v in prof.items() if v[1]},
        "roofline": {"bound": "hbm", "kernel": f"solve_kernel<{args.prec}>", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "algorithmic_bytes_per_launch": nbytes, "launches": launches,
                     "launch_seconds_mean": float(np.sum(kernel_s)) / launches, "traffic": None},
        "cpu_baseline": cpu,
    }
    traffic, tsrc = profiled_traffic(args.workload, args.prec)
    out["roofline"]["traffic"] = traffic
    out["roofline"]["traffic_source"] = tsrc
    if traffic:
        out["roofline"]["traffic_over_algorithmic"] = traffic / nbytes
    if args.copy_calibration:
        xc = torch.ones(1 << 26, device="cuda", dtype=torch.float32)
        yc = torch.empty_like(xc)
        torch.mul(xc, 1.0, out=yc)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = 4 * (1 << 26)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
