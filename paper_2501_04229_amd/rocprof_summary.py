"""Summarise a rocprofv3 results database as Markdown.

    python -m paper_2501_04229_amd.rocprof_summary RESULTS.db [--kernel SUBSTR] [--min-ms MS]
           [--copy-bytes BYTES]

Kernel-trace databases: a per-kernel table (calls, total, mean) and, for the
kernels whose name contains SUBSTR, the launches longer than MS milliseconds
with their mean duration (the statistic bench.py reports for its timed
launches).  Counter databases (--pmc): per-dispatch counter values of those
kernels; with --copy-bytes, the value a counter reads for the largest
elementwise copy dispatch divided by the bytes that copy moves gives the
scale factor from counter units to bytes.
"""
from __future__ import annotations

import argparse
import sqlite3
import statistics


def kernel_table(c, limit=12):
    rows = c.execute("select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
    out = ["| kernel | calls | total ms | mean ms | % |", "|---|---|---|---|---|"]
    for name, calls, tot, avg, pct in rows[:limit]:
        # top_kernels reports microseconds
        out.append(f"| `{name[:110]}` | {calls} | {tot / 1e3:.3f} | {avg / 1e3:.4f} | {pct:.2f} |")
    return "\n".join(out)


def launches(c, substr, min_ms):
    # kernels reports nanoseconds
    rows = c.execute("select name, duration, grid_x, workgroup_x, vgpr_count from kernels where name like ? "
                     "order by start", (f"%{substr}%",)).fetchall()
    long_ = [r for r in rows if r[1] / 1e6 >= min_ms]
    out = [f"launches of kernels matching `{substr}`: {len(rows)}; at least {min_ms} ms: {len(long_)}"]
    if long_:
        d = [r[1] / 1e6 for r in long_]
        out.append(f"mean of those: {statistics.mean(d):.3f} ms (min {min(d):.3f}, max {max(d):.3f}); "
                   f"grid {long_[0][2]} threads, block {long_[0][3]}, {long_[0][4]} VGPRs")
        out.append("durations (ms): " + ", ".join(f"{v:.3f}" for v in d))
    return "\n".join(out)


def counters(c, substr, copy_bytes):
    rows = c.execute("select dispatch_id, kernel_name, counter_name, value from counters_collection "
                     "order by dispatch_id").fetchall()
    by = {}
    for did, name, cn, v in rows:
        by.setdefault((did, name), {})[cn] = by.get((did, name), {}).get(cn, 0.0) + v
    out = []
    scale = {}
    if copy_bytes:
        copies = [(k, v) for k, v in by.items() if "elementwise" in k[1] or "copy" in k[1].lower()]
        if copies:
            for cn in {cn for _, v in copies for cn in v}:
                best = max(v.get(cn, 0.0) for _, v in copies)
                if best > 0:
                    scale[cn] = copy_bytes / best
            out.append("copy calibration (bytes per counter unit): " +
                       ", ".join(f"{k} {v:.1f}" for k, v in sorted(scale.items())))
    for (did, name), vals in by.items():
        if substr in name:
            cells = []
            for cn, v in sorted(vals.items()):
                cell = f"{cn} = {v:.4g}"
                if cn in scale:
                    cell += f" ({v * scale[cn] / 1e9:.3f} GB)"
                cells.append(cell)
            out.append(f"dispatch {did} `{name[:80]}`: " + ", ".join(cells))
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("--kernel", default="solve_kernel")
    ap.add_argument("--min-ms", type=float, default=0.0)
    ap.add_argument("--copy-bytes", type=float, default=0.0)
    a = ap.parse_args()
    c = sqlite3.connect(a.db)
    views = {r[0] for r in c.execute("select name from sqlite_master")}
    has_trace = c.execute("select count(*) from kernels").fetchone()[0] > 0 if "kernels" in views else False
    has_pmc = c.execute("select count(*) from counters_collection").fetchone()[0] > 0 \
        if "counters_collection" in views else False
    if has_trace and "top_kernels" in views:
        print(kernel_table(c))
        print()
        print(launches(c, a.kernel, a.min_ms))
    if has_pmc:
        print(counters(c, a.kernel, a.copy_bytes))


if __name__ == "__main__":
    main()
