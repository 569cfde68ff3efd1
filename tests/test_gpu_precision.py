"""GPU: the precision triples (u_r, u, u_f) of the Section 4.1 precision study (Table 3d).

What the paper's table fixes, checked on a 3-D convection-diffusion system
(the table's matrix family; the paper prints no size, omega or tolerance):
  - double outer precisions (u = u_f = double) reach the double floor whatever u_r is;
  - a single-precision residual (u_f = single) stalls near the single floor, with half
    or single inner solves, however many sweeps run;
  - the solution satisfies the forward-error bound of its residual.
Every residual here is recomputed in double by the CPU oracle.
"""
import math

import numpy as np
import pytest

import gadi_inputs as gi
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2501_04229_amd as gadi  # noqa: E402

N_GRID = 24


@pytest.fixture(scope="module")
def system():
    A = gi.convdiff(N_GRID, 3, 20.0)
    xs, b = gi.rhs_for(A, "uniform", 3)
    return A, b, xs, gadi.System(A), oracle.OracleSystem(A)


def _true_relres(o, A, b, x):
    return float(np.linalg.norm(b - o.spmv("A", x)) / np.linalg.norm(b))


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
def test_double_outer_precision_reaches_the_double_floor(system, prec):
    A, b, xs, g, o = system
    eps = 1e-6 if prec == "fp64" else None
    x, info = g.solve(b, 0.5, 0.5, tol=1e-12, prec=prec, eps_inner=eps, maxit_outer=3000)
    assert info["status"] == gadi.OK, info
    assert _true_relres(o, A, b, x) <= 1.0000001e-12
    lmin = 3 * (2.0 - 2.0 * math.cos(math.pi / (N_GRID + 1)))
    assert np.linalg.norm(x - xs) <= np.linalg.norm(b - o.spmv("A", x)) / lmin * 1.0000001


@pytest.mark.parametrize("prec", ["h-d-s", "h-s-s", "s-s-s"])
def test_single_residual_stalls_at_the_single_floor(system, prec):
    A, b, xs, g, o = system
    x, info = g.solve(b, 0.5, 0.5, tol=1e-13, prec=prec, maxit_outer=300, history=True)
    assert info["status"] == gadi.EMAXIT, info
    h = g.history
    assert len(h) == 301 and np.all(np.isfinite(h))
    # the computed residual cannot fall far below the single unit roundoff ...
    assert h.min() > 1e-9, h.min()
    # ... but the iteration does converge to that floor
    assert h.min() < 1e-4, h.min()
    # and the true (double) residual of the returned solution sits at the same floor
    rel = _true_relres(o, A, b, x)
    assert 1e-9 < rel < 1e-4, rel


def test_single_solution_is_returned_in_double(system):
    """u = single keeps x in fp32 on the device; the caller still gets doubles, and a warm
    start from them continues where the previous solve stopped."""
    A, b, xs, g, o = system
    x1, i1 = g.solve(b, 0.5, 0.5, tol=1e-13, prec="s-s-s", maxit_outer=20)
    assert x1.dtype == np.float64
    assert np.array_equal(x1, x1.astype(np.float32).astype(np.float64))
    rel1 = _true_relres(o, A, b, x1)
    assert rel1 < 0.5
    x2, i2 = g.solve(b, 0.5, 0.5, tol=1e-13, prec="s-s-s", maxit_outer=3, x0=x1)
    assert i2["outer_sweeps"] == 3
    assert _true_relres(o, A, b, x2) < rel1


def test_precision_study_modes_reject_the_batched_sweep(system):
    A, b, xs, g, o = system
    with pytest.raises(gadi.GadiError):
        gadi.solve_batched([g], [b], [0.5], [0.5], prec="h-d-s")
