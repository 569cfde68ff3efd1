"""Host logic of solve_auto (the default judges the prediction), on a stand-in system whose
solves contract the residual at a fixed rate per parameter pair (no GPU)."""
import math
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2501_04229_amd import predictor as pr  # noqa: E402
import paper_2501_04229_amd as gadi  # noqa: E402


class FakeSystem:
    """RES after k sweeps = rate^k from x = 0 (a warm start continues the sequence);
    `work_per_sweep` phases per sweep; `fail` parameter pairs overflow at once."""

    def __init__(self, rates, work_per_sweep, fail=()):
        self.rates, self.wps, self.fail = rates, work_per_sweep, set(fail)
        self.history = None
        self.calls = []

    def features(self, dim, grid, beta):
        return np.zeros(8, np.float32)

    def solve(self, b, alpha, omega, tol=1e-10, x0=None, maxit_outer=20000, history=False, **kw):
        key = (alpha, omega)
        self.calls.append((key, maxit_outer, x0 is not None))
        if key in self.fail:
            self.history = np.zeros(0) if history else self.history
            return np.zeros(3), {"status": gadi.EOVERFLOW16, "outer_sweeps": 0, "inner_H": 1, "inner_S": 0,
                                 "seconds": 1e-3, "relres": float("nan")}
        start = 1.0 if x0 is None else float(x0[0])
        rate = self.rates[key]
        need = math.inf if tol <= 0 else max(0, math.ceil(math.log(tol) / math.log(rate)))
        k = min(need, maxit_outer)
        res = rate ** k
        if history:
            self.history = rate ** np.arange(k + 1)
        x = np.full(3, start * res)
        st = gadi.OK if k == need else gadi.EMAXIT
        w = self.wps[key]
        return x, {"status": st, "outer_sweeps": k, "inner_H": int(w * k) - 5 * k, "inner_S": 0,
                   "seconds": 1e-4 * k, "relres": res}


class ConstPredictor:
    def __init__(self, a, w):
        self.a, self.w = a, w

    def predict(self, f):
        return self.a, self.w


A = type("A", (), {"dim": 3, "grid": 8, "beta": (1.0, 1.0, 1.0)})()


def test_faster_prediction_is_kept():
    s = FakeSystem({(0.2, 0.3): 0.80, (0.5, 0.5): 0.95}, {(0.2, 0.3): 20, (0.5, 0.5): 20})
    x, info, used = pr.solve_auto(s, A, None, ConstPredictor(0.2, 0.3), tol=1e-10)
    assert used == "mlp" and info["status"] == gadi.OK and info["fell_back"] == 0


def test_prediction_over_the_judges_budget_is_rejected_and_the_default_continues_warm():
    """The default needs 219 sweeps x 20 phases; the prediction (rate 0.97) may spend that much,
    has not converged by then, and the default finishes from its iterate."""
    s = FakeSystem({(5.0, 0.5): 0.97, (0.5, 0.5): 0.90}, {(5.0, 0.5): 20, (0.5, 0.5): 20})
    x, info, used = pr.solve_auto(s, A, None, ConstPredictor(5.0, 0.5), tol=1e-10, judge="measure")
    assert used == "default" and info["fell_back"] == 1 and info["status"] == gadi.OK
    assert info["guard"]["judge_work"] == 219 * 20 and info["guard"]["budget_sweeps"] == 219 - 32
    # the judge's solve, the probe, the continuation up to the budget, the default from the iterate
    assert [c[0] for c in s.calls] == [(0.5, 0.5), (5.0, 0.5), (5.0, 0.5), (0.5, 0.5)]
    assert s.calls[2][1] == 219 - 32 and s.calls[3][2]
    assert info["guard_seconds"] > 0
    # the judge is cached on the handle: no second default solve, no guard time
    s.calls.clear()
    x, info, used = pr.solve_auto(s, A, None, ConstPredictor(5.0, 0.5), tol=1e-10, judge="measure")
    assert [c[0] for c in s.calls] == [(5.0, 0.5), (5.0, 0.5), (0.5, 0.5)] and info["guard_seconds"] == 0.0


def test_cheaper_per_sweep_prediction_is_kept_despite_more_sweeps():
    """Work, not sweeps, decides: more sweeps at a third of the work per sweep fit the budget."""
    s = FakeSystem({(0.3, 0.5): 0.92, (0.5, 0.5): 0.90}, {(0.3, 0.5): 10, (0.5, 0.5): 30})
    x, info, used = pr.solve_auto(s, A, None, ConstPredictor(0.3, 0.5), tol=1e-10, judge=219 * 30)
    assert used == "mlp" and info["status"] == gadi.OK


def test_failed_prediction_restarts_the_default_from_zero_and_caches_the_judge():
    s = FakeSystem({(0.5, 0.5): 0.9}, {(0.5, 0.5): 20}, fail=[(1e-3, 0.5)])
    x, info, used = pr.solve_auto(s, A, None, ConstPredictor(1e-3, 0.5), tol=1e-10)
    assert used == "default" and info["status"] == gadi.OK
    assert s.calls[-1] == ((0.5, 0.5), 20000, False)
    assert list(s._default_work.values()) == [219 * 20]


def test_without_a_judge_a_stalled_prediction_is_replaced():
    """No cached judge: a probe whose fitted rate cannot reach tol within the sweep limit hands
    over to the default."""
    s = FakeSystem({(7.0, 0.5): 0.9995, (0.5, 0.5): 0.9}, {(7.0, 0.5): 20, (0.5, 0.5): 20})
    x, info, used = pr.solve_auto(s, A, None, ConstPredictor(7.0, 0.5), tol=1e-10, maxit_outer=5000)
    assert used == "default" and info["status"] == gadi.OK
