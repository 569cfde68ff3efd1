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

# (threads per block, blocks per compute unit, Chronopoulos-Gear inner solves)
SHAPES = [(1024, 1, 1), (1024, 1, 0), (512, 1, 1)]


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


@pytest.mark.parametrize("shape", SHAPES, ids=[f"{b}x{c}_fused{f}" for b, c, f in SHAPES])
def test_solve_parity_multi_tile(big, shape, monkeypatch):
    A, b, o, xref, tol = big
    block, per_cu, fused = shape
    monkeypatch.setenv("GADI_SOLVE_BLOCK", str(block))
    monkeypatch.setenv("GADI_BLOCKS_PER_CU", str(per_cu))
    monkeypatch.setenv("GADI_SOLVE_FUSED", str(fused))
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


def test_solve_auto_parity_multi_tile(big, monkeypatch):
    """The bench's path: features, MLP prediction, guarded probe and continuation."""
    from paper_2501_04229_amd import predictor as pr
    A, b, o, xref, tol = big
    monkeypatch.setenv("GADI_SOLVE_BLOCK", "1024")
    monkeypatch.setenv("GADI_BLOCKS_PER_CU", "1")
    monkeypatch.setenv("GADI_SOLVE_FUSED", "1")
    g = gadi.System(A)
    bd = torch.from_numpy(b).cuda()
    x, info, used = pr.solve_auto(g, A, bd, pr.load(), tol=tol)
    torch.cuda.synchronize()
    _check_shape(g, 1024)
    _check_solution(x.cpu().numpy(), info, b, o, xref, tol)
    g.close()
