"""The allocation-free entry point against gadi_ir_solve (same kernels, same launch shape:
identical iterates), two calls in a row on the shared scratch array, the second on a smaller
system, plus the size limit and the argument rules."""
import ctypes

import numpy as np
import pytest

import gadi_inputs as gi

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2501_04229_amd as gadi  # noqa: E402


def _pair(A, seed, prec, tol, eps):
    g = gadi.System(A)
    xs, b = gi.rhs_for(A, "uniform", seed)
    bd = torch.from_numpy(b).cuda()
    # the normal entry point first: it tunes the launch shape the allocation-free call reuses
    xr, ir = g.solve(bd, 0.3, 0.4, tol=tol, prec=prec, eps_inner=eps)
    x = torch.zeros_like(bd)
    info = g.solve_noalloc(bd, x, 0.3, 0.4, tol=tol, prec=prec, eps_inner=eps)
    torch.cuda.synchronize()
    return g, xr, ir, x, info


@pytest.mark.parametrize("prec,eps", [("fp16", None), ("fp64", 1e-6)])
def test_noalloc_matches_the_allocating_solve_twice(prec, eps):
    print(f"# noalloc {prec}: 3-D 40^3 then 2-D 50^2", flush=True)
    for A, seed in ((gi.convdiff(40, 3, (10.0, 30.0, 2.0)), 3), (gi.convdiff(50, 2, 20.0), 4)):
        g, xr, ir, x, info = _pair(A, seed, prec, 1e-10, eps)
        assert ir["status"] == gadi.OK and info["status"] == gadi.OK, (ir, info)
        assert info["outer_sweeps"] == ir["outer_sweeps"] and info["inner_H"] == ir["inner_H"]
        assert info["inner_S"] == ir["inner_S"] and info["relres"] == ir["relres"]
        # same kernel, same launch shape, deterministic reductions: the same iterates
        assert torch.equal(x, xr), float((x - xr).abs().max())
        g.close()


def test_noalloc_rules_and_size_limit():
    A = gi.convdiff(12, 3, 5.0)
    g = gadi.System(A)
    xs, b = gi.rhs_for(A, "uniform", 1)
    bd = torch.from_numpy(b).cuda()
    x = torch.zeros_like(bd)
    for prec in ("fp32", "fp8", "h-d-s"):
        assert g.solve_noalloc(bd, x, prec=prec)["status"] == gadi.EINVAL
    L = gadi.lib()
    o = gadi.options("fp16", on_device=False)
    info = gadi.SolveInfo()
    assert L.gadi_ir_solve_noalloc(g.handle, ctypes.c_void_p(bd.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                   0.5, 0.5, 1e-10, ctypes.byref(o), ctypes.byref(info)) == gadi.EINVAL
    # 150^3 pads to 3,375,104 rows: beyond the 2,573,753-row scratch array, rejected before any work
    big = gi.convdiff(150, 3, 1.0)
    gb = gadi.System(big)
    bb = torch.zeros(big.n, dtype=torch.float64, device="cuda")
    xb = torch.zeros_like(bb)
    assert gb.solve_noalloc(bb, xb)["status"] == gadi.ENOMEM
    # a solve after the rejection still works
    info = g.solve_noalloc(bd, x, tol=1e-8)
    assert info["status"] == gadi.OK, info
