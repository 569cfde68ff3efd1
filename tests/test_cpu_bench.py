"""Host logic of bench.py (no GPU): the algorithmic byte model behind
roofline.achieved, the traffic summary's staleness rule, the copy-calibrated
counter summaries that give roofline.traffic, and the one-GPU rule."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

# 3-D 128^3 stencil layout: N rows, 6N - 6 n^2 off-diagonal entries, all in diagonal-style slices
N = 128 ** 3
L = {"n": N, "nnz_off": 6 * N - 6 * 128 ** 2, "explicit_entries": 0}


def test_linear_in_the_iteration_counts():
    f = lambda s, h, c, l=1: bench.solve_bytes("fp16", L, s, h, c, l)
    base = f(0, 0, 0, 0)
    assert base == 0.0
    one_res = f(0, 0, 0, 1)
    per_sweep = f(1, 0, 0, 0)
    per_cg = f(0, 1, 0, 0)
    per_cgne = f(0, 0, 1, 0)
    assert f(10, 20, 30, 2) == pytest.approx(2 * one_res + 10 * per_sweep + 20 * per_cg + 30 * per_cgne)
    # a launch evaluates one residual more than it corrects: the residual is in every sweep too
    assert per_sweep > one_res


def test_magnitudes_of_one_unit():
    zo = L["nnz_off"]
    # residual: double A (values of the off-diagonals and the diagonal), x, b, the scaled output
    assert bench.solve_bytes("fp16", L, 0, 0, 0, 1) == 8 * (zo + N) + 22 * N
    # fp16 CG step: the operator once (values + diagonal) and eight half-precision vector accesses
    assert bench.solve_bytes("fp16", L, 0, 1, 0, 0) == 2 * (zo + N) + 16 * N
    # a CGNE step applies S twice
    assert bench.solve_bytes("fp16", L, 0, 0, 1, 0) == 2 * (2 * zo + 8 * N)


def test_precision_and_explicit_columns():
    e = bench.solve_bytes("fp8", L, 5, 50, 20)
    a = bench.solve_bytes("fp16", L, 5, 50, 20)
    # E4M3 values save one byte per off-diagonal entry in every inner product (CG, two per CGNE, update)
    assert a - e == L["nnz_off"] * (50 + 2 * 20 + 5)
    b = bench.solve_bytes("fp32", L, 5, 50, 20)
    c = bench.solve_bytes("fp64", L, 5, 50, 20)
    assert a < b < c
    L2 = dict(L, explicit_entries=1000)
    # each product reads a 4-byte column per explicit entry: residual, CG, two per CGNE, the update's S product
    d = bench.solve_bytes("fp16", L2, 1, 1, 1, 1) - bench.solve_bytes("fp16", L, 1, 1, 1, 1)
    assert d == 4 * 1000 * (2 + 1 + 2 + 1)


def test_stale_traffic_summary_is_ignored(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.profiled_traffic("w", "fp16")[0] is None
    f = prof / "solve_kernel_fp16_w_traffic.md"
    import paper_2501_04229_amd.rocprof_summary as rs
    good = rs.source_hash(ROOT)
    monkeypatch.setattr(rs, "source_hash", lambda root: good)
    f.write_text(f"traffic_bytes_per_launch: 1.5e+10\nsource_sha256: {good}\n")
    assert bench.profiled_traffic("w", "fp16")[0] == 1.5e10
    f.write_text("traffic_bytes_per_launch: 1.5e+10\nsource_sha256: 1234\n")
    assert bench.profiled_traffic("w", "fp16")[0] is None


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "single" in (r.stdout + r.stderr).lower()


def test_survey_byte_model_per_unit():
    """The CSR per-unit figures: residual 12 z + 22 N, fp16 CG step 6 z + 16 N, CGNE step
    2 (6 z_s + 8 N), update 18 N (z with the diagonal, z_s without)."""
    n = 1000
    z, zs = 7 * n - 600, 6 * n - 600
    f = lambda s, h, c, l=1: bench.survey_bytes("fp16", z, zs, n, s, h, c, l)
    assert f(0, 0, 0, 1) == 12 * z + 22 * n
    assert f(0, 1, 0, 0) == 6 * z + 16 * n
    assert f(0, 0, 1, 0) == 2 * (6 * zs + 8 * n)
    assert f(1, 0, 0, 0) == 12 * z + 22 * n + 18 * n


def test_parity_tolerance_closed_form():
    """lambda_min of the h^2-scaled Laplacian and the resulting outer tolerance."""
    import math
    import numpy as np
    import gadi_inputs as gi
    A = gi.convdiff(8, 3, 10.0)
    lam = bench.lambda_min_H(A)
    assert lam == pytest.approx(3 * (2 - 2 * math.cos(math.pi / 9)), rel=1e-15)
    xs, b = gi.rhs_for(A, "ones")
    t = bench.parity_tolerance(A, b, xs)
    assert t == min(1e-10, 0.9 * (1e-8 * lam * np.linalg.norm(xs) / np.linalg.norm(b) - 1e-13))


def _counter_db(path, counter, rows):
    """A counter database with the columns the summary reads: rows of
    (dispatch_id, kernel_name, grid_size, workgroup_size, value); a dispatch may
    have several rows (per-instance readings), which add up."""
    import sqlite3
    c = sqlite3.connect(str(path))
    c.execute("create table counters_collection (dispatch_id int, kernel_name text, grid_size int, "
              "workgroup_size int, counter_name text, value real)")
    c.executemany("insert into counters_collection values (?, ?, ?, ?, ?, ?)",
                  [(d, k, g, w, counter, v) for d, k, g, w, v in rows])
    c.commit()
    c.close()
    return str(path)


def test_counter_traffic_is_copy_calibrated(tmp_path):
    """The copy dispatch fixes the bytes per counter unit of each run; the timed launches
    are the `launches` dispatches before the last matching one, and per-(kernel, grid)
    means keep the sizes of one kernel apart."""
    import paper_2501_04229_amd.rocprof_summary as rs
    copy = 1 << 20
    # fetch counter: 1 unit = 2 bytes (the copy reads 2^20 bytes and reads 2^19); write: 1 unit = 4 bytes
    f = _counter_db(tmp_path / "f.db", "FETCH_SIZE", [
        (1, "gadi::solve_kernel<A>", 100, 10, 10e6), (1, "gadi::solve_kernel<A>", 100, 10, 5e6),
        (2, "gadi::solve_kernel<A>", 100, 10, 30e6),
        (3, "gadi::solve_kernel<A>", 200, 10, 70e6),
        (4, "gadi::solve_kernel<A>", 200, 10, 1000e6),
        (5, "elementwise_kernel<copy>", 1, 1, copy / 2)])
    w = _counter_db(tmp_path / "w.db", "WRITE_SIZE", [
        (1, "gadi::solve_kernel<A>", 100, 10, 1e6), (2, "gadi::solve_kernel<A>", 100, 10, 3e6),
        (3, "gadi::solve_kernel<A>", 200, 10, 5e6), (4, "gadi::solve_kernel<A>", 200, 10, 500e6),
        (5, "elementwise_kernel<copy>", 1, 1, copy / 4)])
    out = rs.traffic(f, w, "solve_kernel", 2, copy)
    # timed launches: dispatches 2 and 3 (the last matching one, 4, is the reference solve)
    # fetch (30 + 70) * 2 = 200 MB, write (3 + 5) * 4 = 32 MB, over 2 launches
    assert "traffic_bytes_per_launch: 1.160000e+08" in out
    table = rs.traffic_by_grid(f, w, "solve_kernel", copy)
    rows = {ln.split("|")[2].strip(): ln for ln in table.splitlines() if ln.startswith("| `")}
    # grid 100 (MB columns): dispatch 1 sums its two readings (15e6 units) and dispatch 2 reads 30e6: mean 22.5e6
    # units = 45 MB; writes (1 + 3) / 2 = 2e6 units = 8 MB
    cells = [x.strip() for x in rows["100"].split("|")]
    assert cells[4] == "2" and float(cells[5]) == 45.0 and float(cells[6]) == 8.0
    cells = [x.strip() for x in rows["200"].split("|")]
    assert float(cells[5]) == (70 + 1000) / 2 * 2 and float(cells[7]) == 1070.0 + (5 + 500) / 2 * 4
