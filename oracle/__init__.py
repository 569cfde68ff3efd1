"""CPU oracle for GADI-IR -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its binding) never
imports it and shares no code with it.

Contents:
  * `OracleSystem`: ctypes binding of the plain FP64 C oracle in
    gadi_oracle.c (HSS splitting, SpMV, GADI-IR with CG / CGNE inner solves,
    Gershgorin bounds).
  * `dense`: dense numpy forms for tiny grids (exact-inner GADI, the
    Theorem 1 iteration matrix, closed-form spectra).
  * `mlp`: a float64 numpy multilayer perceptron with hand-derived gradients.
  * `features`: the predictor's input features computed from the oracle's
    splitting.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gadi_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

STATUS = {0: "ok", 1: "einval", 2: "enotspd", 4: "ediverged", 5: "emaxit", 7: "enomem"}


def build(force: bool = False, plant: int = 0) -> str:
    """Compile the C oracle with gcc (plain -O2, no FMA contraction, OpenMP).

    plant != 0 builds a deliberately wrong variant (for the test that shows
    the pins catch planted mistakes) under a separate file name."""
    lib = _LIB if plant == 0 else _LIB.replace(".so", "_plant%d.so" % plant)
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
        tmp = lib + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-shared", "-fPIC", "-std=c11", "-DORACLE_PLANT=%d" % plant, _SRC,
                               "-o", tmp, "-lm"])
        os.replace(tmp, lib)
    return lib


_lib_handle = None
_plant_handles = {}


def _load(path):
    lib = ctypes.CDLL(path)
    _declare(lib)
    return lib


def _lib(plant: int = 0):
    global _lib_handle
    if plant:
        if plant not in _plant_handles:
            _plant_handles[plant] = _load(build(plant=plant))
        return _plant_handles[plant]
    if _lib_handle is None:
        _lib_handle = _load(build())
    return _lib_handle


def _declare(lib):
    if True:
        P = ctypes.POINTER
        i32p, f64p, i64p = P(ctypes.c_int32), P(ctypes.c_double), P(ctypes.c_int64)
        lib.oracle_setup.restype = ctypes.c_void_p
        lib.oracle_setup.argtypes = [ctypes.c_int, i32p, i32p, f64p]
        lib.oracle_free.argtypes = [ctypes.c_void_p]
        lib.oracle_split_ok.argtypes = [ctypes.c_void_p]
        lib.oracle_split_nnz.restype = ctypes.c_int64
        lib.oracle_split_nnz.argtypes = [ctypes.c_void_p]
        lib.oracle_get_split.argtypes = [ctypes.c_void_p, ctypes.c_int, i32p, i32p, f64p]
        lib.oracle_spmv.argtypes = [ctypes.c_void_p, ctypes.c_int, f64p, f64p]
        lib.oracle_gadi.argtypes = [ctypes.c_void_p, f64p, f64p, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                    ctypes.c_int, P(ctypes.c_int), i64p, i64p, f64p, f64p,
                                    ctypes.c_int]
        lib.oracle_gershgorin.argtypes = [ctypes.c_void_p, f64p]
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_num_threads.argtypes = []
        lib.oracle_set_num_threads.restype = None
        lib.oracle_set_num_threads.argtypes = [ctypes.c_int]


def set_num_threads(n: int) -> None:
    """Threads for the oracle's OpenMP loops (timing only: the results do not depend on it)."""
    _lib().oracle_set_num_threads(int(n))


def num_threads() -> int:
    """OpenMP threads the oracle's loops use."""
    return int(_lib().oracle_num_threads())


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


class OracleSystem:
    """A system prepared by the C oracle: A, H = (A+A^T)/2, S = (A-A^T)/2."""

    def __init__(self, A, plant: int = 0):
        self._L = _lib(plant)
        self.n = int(A.n)
        self._rp = np.ascontiguousarray(A.row_ptr, dtype=np.int32)
        self._col = np.ascontiguousarray(A.col, dtype=np.int32)
        self._val = np.ascontiguousarray(A.val, dtype=np.float64)
        self.meta = A
        h = self._L.oracle_setup(self.n, _ptr(self._rp, ctypes.c_int32), _ptr(self._col, ctypes.c_int32),
                                _ptr(self._val, ctypes.c_double))
        if not h:
            raise ValueError("oracle_setup rejected the CSR matrix")
        self._h = ctypes.c_void_p(h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and getattr(self, "_L", None) is not None:
            self._L.oracle_free(h)
            self._h = None

    @property
    def split_ok(self) -> bool:
        return bool(self._L.oracle_split_ok(self._h))

    def split(self, which: str):
        """Return (row_ptr, col, val) of 'H' or 'S'."""
        nnz = self._L.oracle_split_nnz(self._h)
        rp = np.empty(self.n + 1, np.int32)
        col = np.empty(nnz, np.int32)
        val = np.empty(nnz, np.float64)
        self._L.oracle_get_split(self._h, {"H": 1, "S": 2}[which], _ptr(rp, ctypes.c_int32),
                                _ptr(col, ctypes.c_int32), _ptr(val, ctypes.c_double))
        return rp, col, val

    def spmv(self, which: str, x) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.empty(self.n)
        self._L.oracle_spmv(self._h, {"A": 0, "H": 1, "S": 2}[which], _ptr(x, ctypes.c_double),
                           _ptr(y, ctypes.c_double))
        return y

    def gadi(self, b, alpha, omega, tol=1e-10, eps_h=1e-6, eps_s=1e-6, maxit_out=100000,
             maxit_in=100000, x0=None, hist_len=0):
        """Run GADI-IR in double; returns a dict with x, status, sweeps, inner counts, relres."""
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros(self.n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        sweeps = ctypes.c_int(0)
        ih, is_ = ctypes.c_int64(0), ctypes.c_int64(0)
        rel = ctypes.c_double(0.0)
        hist = np.zeros(max(hist_len, 1))
        st = self._L.oracle_gadi(self._h, _ptr(b, ctypes.c_double), _ptr(x, ctypes.c_double),
                                float(alpha), float(omega), float(tol), float(eps_h), float(eps_s),
                                int(maxit_out), int(maxit_in), ctypes.byref(sweeps), ctypes.byref(ih),
                                ctypes.byref(is_), ctypes.byref(rel), _ptr(hist, ctypes.c_double),
                                int(hist_len))
        out = {"x": x, "status": STATUS.get(st, str(st)), "sweeps": sweeps.value,
               "inner_h": ih.value, "inner_s": is_.value, "relres": rel.value}
        if hist_len:
            out["hist"] = hist[: min(hist_len, sweeps.value + 1)]
        return out

    def gershgorin(self) -> np.ndarray:
        out = np.zeros(4)
        self._L.oracle_gershgorin(self._h, _ptr(out, ctypes.c_double))
        return out


def features(A, gersh=None) -> np.ndarray:
    """Predictor features of a convection-diffusion system.

    [ln N, dim, log10 mean(beta), log10 Pe with Pe = max_a beta_a h / 2,
     log10 lambda_min(H), log10 max_i(H_ii + R_i^H), log10 max_i R_i^S, log10 min_i R_i^S]
    with h = 1/(n+1), lambda_min(H) = dim (2 - 2 cos(pi h)) (the smallest
    eigenvalue of the h^2-scaled Laplacian, Section 4.1's symmetric part), R_i
    the off-diagonal absolute row sums of H, S, and the log10 arguments
    floored at 1e-12.
    """
    if gersh is None:
        gersh = OracleSystem(A).gershgorin()
    beta = np.asarray(A.beta, dtype=np.float64)
    h = 1.0 / (A.grid + 1)

    def lg(v):
        return math.log10(max(v, 1e-12))
    return np.array([math.log(A.n), float(A.dim), math.log10(float(beta.mean())),
                     lg(float(beta.max()) * h / 2.0), lg(A.dim * (2.0 - 2.0 * math.cos(math.pi * h))),
                     lg(gersh[1]), lg(gersh[2]), lg(gersh[3])])
