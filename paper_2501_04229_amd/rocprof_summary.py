"""Summarise a rocprofv3 results database as Markdown.

    python -m paper_2501_04229_amd.rocprof_summary RESULTS.db [--kernel SUBSTR] [--min-ms MS]
           [--copy-bytes BYTES]
    python -m paper_2501_04229_amd.rocprof_summary --traffic FETCH.db WRITE.db --kernel SUBSTR
           --launches L --copy-bytes BYTES
    python -m paper_2501_04229_amd.rocprof_summary --traffic FETCH.db WRITE.db --kernel SUBSTR --by-grid
           --copy-bytes BYTES

The second form combines a FETCH_SIZE run and a WRITE_SIZE run of the same
command: the dispatches of the kernels matching SUBSTR, taken in order, end
with the L launches of the timed step followed by one more launch (the
reference solve bench.py runs after its timed steps); their counter values,
scaled to bytes by the copy calibration of each run, give the HBM bytes per
launch.  The output carries a machine-readable line with that figure and the
source hash bench.py checks before it reports the figure.

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


def by_grid(c, substr):
    """Launches of kernels matching substr grouped by (kernel, launch grid): calls and mean duration, so that
    runs of one kernel at several problem sizes in one trace stay apart."""
    rows = c.execute("select name, grid_x * grid_y * grid_z, workgroup_x, count(*), avg(duration), sum(duration) "
                     "from kernels where name like ? group by name, grid_x, grid_y, grid_z, workgroup_x "
                     "order by grid_x * grid_y * grid_z, sum(duration) desc", (f"%{substr}%",)).fetchall()
    out = ["| kernel | grid threads | block | calls | mean us | total ms |", "|---|---|---|---|---|---|"]
    for name, grid, block, calls, avg, tot in rows:
        short = name.split("(")[0].replace("void ", "")
        out.append(f"| `{short}` | {grid} | {block} | {calls} | {avg / 1e3:.1f} | {tot / 1e6:.3f} |")
    return "\n".join(out)


def launches(c, substr, min_ms, timed=0):
    # kernels reports nanoseconds
    rows = c.execute("select name, duration, grid_x, workgroup_x, vgpr_count from kernels where name like ? "
                     "order by start", (f"%{substr}%",)).fetchall()
    if timed:
        # the timed launches: the `timed` launches before the last one (bench.py's reference solve)
        sel = rows[-(timed + 1):-1]
        d = [r[1] / 1e6 for r in sel]
        out = [f"launches of kernels matching `{substr}`: {len(rows)}; timed launches (the {timed} before the last): "
               f"mean {statistics.mean(d):.3f} ms, total {sum(d):.3f} ms; grid {sel[0][2]} threads, block {sel[0][3]}, "
               f"{sel[0][4]} VGPRs",
               "timed durations (ms): " + ", ".join(f"{v:.3f}" for v in d),
               "all durations (ms): " + ", ".join(f"{r[1] / 1e6:.3f}" for r in rows)]
        return "\n".join(out)
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


def dispatch_counters(c, substr, counter):
    """[(dispatch_id, kernel_name, value)] of one counter, in dispatch order."""
    rows = c.execute("select dispatch_id, kernel_name, value from counters_collection where counter_name = ? "
                     "order by dispatch_id", (counter,)).fetchall()
    by = {}
    for did, name, v in rows:
        key = (did, name)
        by[key] = by.get(key, 0.0) + v
    return [(d, n, v) for (d, n), v in sorted(by.items())]


def copy_scale(c, counter, copy_bytes):
    """Bytes per counter unit: copy_bytes over the counter's reading for the largest elementwise copy."""
    vals = [v for _, n, v in dispatch_counters(c, "", counter) if "elementwise" in n or "copy" in n.lower()]
    return copy_bytes / max(vals) if vals else float("nan")


def traffic(fetch_db, write_db, substr, launches, copy_bytes):
    out = []
    tot = 0.0
    per = []
    for db, counter in ((fetch_db, "FETCH_SIZE"), (write_db, "WRITE_SIZE")):
        c = sqlite3.connect(db)
        scale = copy_scale(c, counter, copy_bytes)
        rows = [r for r in dispatch_counters(c, substr, counter) if substr in r[1]]
        step = rows[-(launches + 1):-1]
        b = [v * scale for _, _, v in step]
        per.append(b)
        tot += sum(b)
        out.append(f"{counter}: {scale:.1f} bytes per counter unit (copy of {copy_bytes:.0f} bytes); "
                   f"timed launches " + ", ".join(f"dispatch {d}: {v * scale / 1e9:.3f} GB" for d, _, v in step))
    out.append(f"per launch: fetch {sum(per[0]) / launches / 1e9:.3f} GB, write {sum(per[1]) / launches / 1e9:.3f} GB")
    out.append(f"traffic_bytes_per_launch: {tot / launches:.6e}")
    return "\n".join(out)


def traffic_by_grid(fetch_db, write_db, substr, copy_bytes):
    """Mean HBM bytes per dispatch of each (kernel, launch grid, block) matching substr, from a FETCH_SIZE and a
    WRITE_SIZE counter run, each scaled by its own copy calibration."""
    import sqlite3
    per = {}
    scales = []
    for db, counter in ((fetch_db, "FETCH_SIZE"), (write_db, "WRITE_SIZE")):
        c = sqlite3.connect(db)
        scale = copy_scale(c, counter, copy_bytes)
        scales.append(f"{counter} {scale:.1f}")
        rows = c.execute("select dispatch_id, kernel_name, grid_size, workgroup_size, value from counters_collection "
                         "where counter_name = ? and kernel_name like ?", (counter, f"%{substr}%")).fetchall()
        by = {}
        for did, name, grid, wg, v in rows:
            key = (name.split("(")[0].replace("void ", ""), grid, wg)
            by.setdefault(key, {}).setdefault(did, 0.0)
            by[key][did] += v
        for key, d in by.items():
            per.setdefault(key, {})[counter] = (len(d), sum(d.values()) / len(d) * scale)
    out = ["copy calibration (bytes per counter unit): " + ", ".join(scales), "",
           "| kernel | grid threads | block | dispatches | fetch MB | write MB | total MB |", "|---|---|---|---|---|---|---|"]
    for (name, grid, wg), v in sorted(per.items(), key=lambda kv: (kv[0][1], kv[0][0])):
        nd, f = v.get("FETCH_SIZE", (0, float("nan")))
        _, w = v.get("WRITE_SIZE", (0, float("nan")))
        out.append(f"| `{name}` | {grid} | {wg} | {nd} | {f / 1e6:.2f} | {w / 1e6:.2f} | {(f + w) / 1e6:.2f} |")
    return "\n".join(out)


def source_hash(root):
    """sha256 over the sources that fix the timed launches: libgadi's sources, the
    predictor (weights and solve_auto) and the workload generator."""
    import glob
    import hashlib
    import os
    files = sorted(glob.glob(os.path.join(root, "paper_2501_04229_amd", "csrc", "*")))
    files += [os.path.join(root, "paper_2501_04229_amd", "predictor", "__init__.py"),
              os.path.join(root, "paper_2501_04229_amd", "predictor", "mlp_weights.npz"),
              os.path.join(root, "gadi_inputs", "convdiff.py")]
    h = hashlib.sha256()
    for f in files:
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()


def main():
    import os
    ap = argparse.ArgumentParser()
    ap.add_argument("db", nargs="?")
    ap.add_argument("--traffic", nargs=2, metavar=("FETCH_DB", "WRITE_DB"))
    ap.add_argument("--launches", type=int, default=1)
    ap.add_argument("--timed", type=int, default=0,
                    help="kernel trace: report the TIMED launches before the last matching one")
    ap.add_argument("--kernel", default="solve_kernel")
    ap.add_argument("--min-ms", type=float, default=0.0)
    ap.add_argument("--copy-bytes", type=float, default=0.0)
    ap.add_argument("--by-grid", action="store_true",
                    help="group the matching launches by kernel and launch grid (kernel trace: durations; "
                         "with --traffic: mean HBM bytes per dispatch)")
    a = ap.parse_args()
    if a.traffic and a.by_grid:
        print(traffic_by_grid(a.traffic[0], a.traffic[1], a.kernel, a.copy_bytes))
        return
    if a.traffic:
        print(traffic(a.traffic[0], a.traffic[1], a.kernel, a.launches, a.copy_bytes))
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        print(f"source_sha256: {source_hash(root)}")
        return
    c = sqlite3.connect(a.db)
    views = {r[0] for r in c.execute("select name from sqlite_master")}
    has_trace = c.execute("select count(*) from kernels").fetchone()[0] > 0 if "kernels" in views else False
    has_pmc = c.execute("select count(*) from counters_collection").fetchone()[0] > 0 \
        if "counters_collection" in views else False
    if has_trace and a.by_grid:
        print(by_grid(c, a.kernel))
        return
    if has_trace and "top_kernels" in views:
        print(kernel_table(c))
        print()
        print(launches(c, a.kernel, a.min_ms, a.timed))
    if has_pmc:
        print(counters(c, a.kernel, a.copy_bytes))


if __name__ == "__main__":
    main()
