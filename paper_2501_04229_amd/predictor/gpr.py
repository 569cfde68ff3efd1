"""The paper's size-based predictor (Section 3.3): Gaussian-process regression
of log10 alpha on log2 n over small systems of one structure, extrapolated to
large n.  The regression runs in libgadi (gadi_gpr_*); this module marshals
arguments and implements the paper's retraining loop, in which each predicted
point joins the training set before the next, larger size is predicted.
"""
from __future__ import annotations

import ctypes

import numpy as np

from .. import _check, _track, lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class GPR:
    """y(x) = b0 + b1 x + GP(x) fitted by libgadi (gadi_gpr_fit)."""

    def __init__(self, x, y):
        self._x = np.ascontiguousarray(x, dtype=np.float64)
        self._y = np.ascontiguousarray(y, dtype=np.float64)
        if self._x.shape != self._y.shape or self._x.ndim != 1:
            raise ValueError("x and y must be 1-D arrays of one length")
        h = ctypes.c_void_p()
        _check(lib().gadi_gpr_fit(_dp(self._x), _dp(self._y), len(self._x), ctypes.byref(h)), "gadi_gpr_fit")
        self._h = h
        _track(self)

    def close(self):
        if getattr(self, "_h", None) and lib() is not None:
            lib().gadi_gpr_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def predict(self, xq):
        xq = np.ascontiguousarray(np.atleast_1d(xq), dtype=np.float64)
        mean = np.empty_like(xq)
        sd = np.empty_like(xq)
        _check(lib().gadi_gpr_predict(self._h, _dp(xq), len(xq), _dp(mean), _dp(sd)), "gadi_gpr_predict")
        return mean, sd

    def params(self) -> dict:
        out = np.empty(6)
        _check(lib().gadi_gpr_params(self._h, _dp(out)), "gadi_gpr_params")
        return dict(zip(("b0", "b1", "ell", "sf2", "sn2", "lml"), out.tolist()))


def predict_alpha(sizes, alphas, targets, retrain=True):
    """alpha for each target size from (size, best alpha) training pairs:
    GPR of log10 alpha on log2 n.  With retrain, targets are predicted in
    ascending order and each prediction joins the training set before the
    next.  Returns a list of (size, alpha, sd of log10 alpha)."""
    xs = list(np.log2(np.asarray(sizes, float)))
    ys = list(np.log10(np.asarray(alphas, float)))
    out = []
    for n in sorted(targets):
        g = GPR(np.array(xs), np.array(ys))
        m, s = g.predict(np.log2(float(n)))
        g.close()
        out.append((n, float(10.0 ** m[0]), float(s[0])))
        if retrain:
            xs.append(float(np.log2(n)))
            ys.append(float(m[0]))
    return out


def dichotomy_search(f, lo=-1.5, hi=1.5, coarse=7, delta=0.01, width=0.08):
    """Near-optimal log10 alpha of one small system (Section 3.3 finds the
    training set's alphas by a dichotomy search): f(u) is the cost of a solve
    with alpha = 10^u (infinite for a failed solve).  A coarse scan of `coarse`
    points over [lo, hi] brackets the best scan point by its neighbours; then,
    while the bracket is wider than `width` decades, f is compared at mid -+
    delta and the better half is kept (both halves' inner ends when they tie).
    Returns (u, f(u), evaluations) for the cheapest evaluated point inside the
    final bracket, ties going to the larger alpha; (nan, inf, evaluations) when
    every scan point failed."""
    import math
    cache = {}

    def ev(u):
        key = round(float(u), 9)
        if key not in cache:
            cache[key] = float(f(key))
        return cache[key]

    grid = np.linspace(lo, hi, coarse)
    vals = [ev(u) for u in grid]
    k = int(np.argmin(vals))
    if not math.isfinite(vals[k]):
        return math.nan, math.inf, len(cache)
    a, c = grid[max(k - 1, 0)], grid[min(k + 1, coarse - 1)]
    while c - a > width:
        mid = 0.5 * (a + c)
        fl, fr = ev(mid - delta), ev(mid + delta)
        if fl < fr:
            c = mid + delta
        elif fr < fl:
            a = mid - delta
        else:
            a, c = mid - delta, mid + delta
    inside = {u: v for u, v in cache.items() if a - 1e-9 <= u <= c + 1e-9} or cache
    u_best = min(inside, key=lambda u: (inside[u], -u))
    return u_best, cache[u_best], len(cache)
