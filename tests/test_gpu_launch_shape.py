"""Oracle-solution parity in the launch configuration of the large solves.

At the small parity sizes every block of the persistent solve kernel owns one
row tile, so neither the two-tiles-in-flight row loop nor the XCD remap of
block indices (which needs a block count divisible by 8) runs.  Here a
531,441-row system (3-D, n = 81, 519 tiles of 1024 rows) is solved with launch
shapes that give every block at least two tiles and a block count divisible by
8, in every inner precision and through `solve_auto` with the committed
predictor, and each solution is compared with the oracle's (run to RES 1e-13)
at relative 1e-8, with the FP64 residual recomputed by the oracle.
"""
import os

import numpy as np
import pytest

import gadi_inputs as gi
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2501_04229_amd as gadi  # noqa: E402
from test_gpu_parity import parity_tol  # noqa: E402

# (threads per block, blocks per compute unit, inner-solver form: 0 Hestenes-Stiefel,
# 1 Chronopoulos-Gear, 2 pipelined CG with Craig's CGNE, 3 Hestenes-Stiefel CG with Craig's CGNE)
SHAPES = [(1024, 1, 1), (1024, 1, 0), (512, 1, 1), (1024, 1, 2), (512, 1, 2), (1024, 1, 3), (512, 1, 3)]


@pytest.fixture(scope="module")
def big():
    A = gi.convdiff(81, 3, (30.0, 5.0, 60.0))
    xs, b = gi.rhs_for(A, "uniform", 0)
    o = oracle.OracleSystem(A)
    print(f"# oracle reference at n = {A.n}", flush=True)
    r = o.gadi(b, 0.5, 0.5, tol=1e-13, eps_h=1e-6, eps_s=1e-6)
    assert r["status"] == "ok"
    xref = r["x"]
    return A, b, o, xref, parity_tol(A, b, xref)


def _check_shape(g, block):
    nb, thr = g.solver_blocks()
    ntiles = g.layout()["npad"] // thr
    assert thr == block and nb % 8 == 0 and ntiles >= 2 * nb, (nb, thr, ntiles)


def _check_solution(x, info, b, o, xref, tol):
    assert info["status"] == gadi.OK, info
    rel = np.linalg.norm(b - o.spmv("A", x)) / np.linalg.norm(b)
    assert rel <= tol * 1.0000001, (rel, info)
    err = np.linalg.norm(x - xref) / np.linalg.norm(xref)
    assert err <= 1e-8, (err, tol, info)


@pytest.mark.parametrize("shape", SHAPES, ids=[f"{b}x{c}_form{f}" for b, c, f in SHAPES])
def test_solve_parity_multi_tile(big, shape, monkeypatch):
    A, b, o, xref, tol = big
    block, per_cu, form = shape
    monkeypatch.setenv("GADI_SOLVE_BLOCK", str(block))
    monkeypatch.setenv("GADI_BLOCKS_PER_CU", str(per_cu))
    monkeypatch.setenv("GADI_SOLVE_FORM", str(form))
    g = gadi.System(A)
    bd = torch.from_numpy(b).cuda()
    for prec in ("fp16", "fp32", "fp64", "fp8"):
        print(f"# {shape} {prec}", flush=True)
        eps = 1e-6 if prec == "fp64" else None
        x, info = g.solve(bd, 0.5, 0.5, tol=tol, prec=prec, eps_inner=eps)
        torch.cuda.synchronize()
        _check_shape(g, block)
        _check_solution(x.cpu().numpy(), info, b, o, xref, tol)
    g.close()


@pytest.mark.parametrize("form", [1, 2, 3])
def test_solve_auto_parity_multi_tile(big, form, monkeypatch):
    """The bench's path: features, MLP prediction, guarded probe and continuation."""
    from paper_2501_04229_amd import predictor as pr
    A, b, o, xref, tol = big
    monkeypatch.setenv("GADI_SOLVE_BLOCK", "1024")
    monkeypatch.setenv("GADI_BLOCKS_PER_CU", "1")
    monkeypatch.setenv("GADI_SOLVE_FORM", str(form))
    g = gadi.System(A)
    bd = torch.from_numpy(b).cuda()
    x, info, used = pr.solve_auto(g, A, bd, pr.load(), tol=tol)
    torch.cuda.synchronize()
    _check_shape(g, 1024)
    _check_solution(x.cpu().numpy(), info, b, o, xref, tol)
    g.close()


@pytest.mark.parametrize("form", [0, 2])
def test_barrier_protocols_agree_bitwise(big, form, monkeypatch):
    """The relay, XCC-hierarchical and master-free XCC barriers all combine the blocks' partial
    sums in block order with the same arithmetic, so one launch shape gives bit-identical
    iterates under each of them; each solution also matches the oracle's."""
    A, b, o, xref, tol = big
    monkeypatch.setenv("GADI_SOLVE_BLOCK", "1024")
    monkeypatch.setenv("GADI_BLOCKS_PER_CU", "1")
    monkeypatch.setenv("GADI_SOLVE_FORM", str(form))
    g = gadi.System(A)
    bd = torch.from_numpy(b).cuda()
    runs = {}
    for kind in ("relay", "xcc", "direct"):
        print(f"# barrier {kind} form {form}", flush=True)
        monkeypatch.setenv("GADI_BARRIER", kind)
        x, info = g.solve(bd, 0.5, 0.5, tol=tol, prec="fp16")
        torch.cuda.synchronize()
        _check_shape(g, 1024)
        xh = x.cpu().numpy()
        _check_solution(xh, info, b, o, xref, tol)
        runs[kind] = (xh, (info["outer_sweeps"], info["inner_H"], info["inner_S"]))
    for kind in ("xcc", "direct"):
        assert runs[kind][1] == runs["relay"][1], (kind, runs[kind][1], runs["relay"][1])
        assert np.array_equal(runs[kind][0], runs["relay"][0]), kind
    g.close()


@pytest.mark.parametrize("form", [0, 2])
@pytest.mark.parametrize("prec", ["fp16", "fp64"])
def test_mirrored_pattern_equals_generic_layout(big, form, prec, monkeypatch):
    """The uniform stencil layout reads H and S through their positive offsets only (the entry at
    -d of row i is the one at +d of row i - d, negated for S); the per-slice generic pattern reads
    every stored slot.  Both sum the same values in the same slot order, so the solves agree bit
    for bit."""
    A, b, o, xref, tol = big
    monkeypatch.setenv("GADI_SOLVE_BLOCK", "1024")
    monkeypatch.setenv("GADI_BLOCKS_PER_CU", "1")
    monkeypatch.setenv("GADI_SOLVE_FORM", str(form))
    g = gadi.System(A)
    assert g.layout()["uniform_offsets"] == 6
    bd = torch.from_numpy(b).cuda()
    eps = 1e-6 if prec == "fp64" else None
    runs = []
    for pattern in ("uniform", "generic"):
        if pattern == "generic":
            monkeypatch.setenv("GADI_SOLVE_PATTERN", "generic")
        x, info = g.solve(bd, 0.5, 0.5, tol=tol, prec=prec, eps_inner=eps)
        torch.cuda.synchronize()
        xh = x.cpu().numpy()
        _check_solution(xh, info, b, o, xref, tol)
        runs.append((xh, (info["outer_sweeps"], info["inner_H"], info["inner_S"])))
    assert runs[0][1] == runs[1][1], (runs[0][1], runs[1][1])
    assert np.array_equal(runs[0][0], runs[1][0])
    g.close()
