"""FP8 storage of H and S (GADI_PREC_FP8_IR) against FP16-IR.

    python -m paper_2501_04229_amd.experiments.fp8_study

For the 128^3 and 256^3 convection-diffusion workloads: device time of the
stand-alone (alpha I + H) x products with fp16 and E4M3 values (a replayed
graph of 50 products, best of 3 replays; algorithmic bytes 2 (z_o + N) + 4 N
and z_o + 2 N + 4 N), and FP16 / FP8 solves to RES 1e-10 at the default and
at the predicted parameters of the 128^3 workload.
"""
from __future__ import annotations

import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import gadi_inputs as gi  # noqa: E402
import paper_2501_04229_amd as gadi  # noqa: E402


def graph_time(fn, out, reps=50):
    import torch
    fn()
    torch.cuda.synchronize()
    ref = out.clone()
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gr):
        for _ in range(reps):
            fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(3):
        out.zero_()
        e0.record()
        gr.replay()
        e1.record()
        torch.cuda.synchronize()
        if not torch.equal(out, ref):
            raise RuntimeError("a graph replay of the product differs from the eager call")
        best = min(best, e0.elapsed_time(e1) * 1e-3 / reps)
    return best


def main():
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("the FP8 study runs on the GPU")
    rows = []
    for name in ("convdiff3d_128_beta20", "convdiff3d_256_betaU100"):
        w = gi.workload(name)
        A = w["A"]
        g = gadi.System(A)
        n = A.n
        L = g.layout()
        b = torch.from_numpy(w["b"]).cuda()
        x = torch.rand(n, device="cuda", dtype=torch.float16, generator=torch.Generator("cuda").manual_seed(3))
        y = torch.empty_like(x)
        t16 = graph_time(lambda: g.spmv("H16", x, y, 0.5), y)
        t8 = graph_time(lambda: g.spmv("H8", x, y, 0.5), y)
        by16 = 2.0 * (L["nnz_off"] + n) + 4.0 * L["explicit_entries"] + 4.0 * n
        by8 = 1.0 * L["nnz_off"] + 4.0 * L["explicit_entries"] + 6.0 * n
        row = {"workload": name, "H16_us": t16 * 1e6, "H16_GBs": by16 / t16 / 1e9, "H8_us": t8 * 1e6,
               "H8_GBs": by8 / t8 / 1e9, "solves": []}
        print(f"{name}: H16 {t16 * 1e6:.1f} us ({by16 / t16 / 1e9:.0f} GB/s), H8 {t8 * 1e6:.1f} us "
              f"({by8 / t8 / 1e9:.0f} GB/s)", flush=True)
        for prec in ("fp16", "fp8"):
            for al, om in ((0.5, 0.5), (0.242, 0.321)):
                g.solve(b, al, om, tol=1e-10, prec=prec, maxit_outer=3)
                _, info = g.solve(b, al, om, tol=1e-10, prec=prec)
                row["solves"].append({"prec": prec, "alpha": al, "omega": om, "status": info["status_str"],
                                      "sweeps": info["outer_sweeps"], "seconds": info["seconds"],
                                      "relres": info["relres"]})
                print(f"  {prec} ({al}, {om}): {info['status_str']} {info['outer_sweeps']} sweeps "
                      f"{info['seconds']:.4f} s relres {info['relres']:.2e}", flush=True)
        g.close()
        rows.append(row)
    print(json.dumps({"fp8_study": len(rows)}))


if __name__ == "__main__":
    main()
