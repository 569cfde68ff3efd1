"""GADI-IR on AMD MI355X: thin Python binding of libgadi.so.

Every step of the solver runs in the HIP kernels of libgadi.so; this module
only marshals arguments (numpy arrays for host memory, torch tensors for
device memory and streams) and raises on error statuses.  There is no CPU
fallback: importing fails if the library cannot be loaded.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref

import numpy as np

from . import build as _build

LIB_PATH = _build.LIB

OK, EINVAL, ENOTSPD, EOVERFLOW16, EDIVERGED, EMAXIT, EHIP, ENOMEM, EBARRIER, EPRUNED = range(10)
PREC = {"fp64": 0, "fp16": 1, "fp32": 2, "h-d-s": 3, "h-s-s": 4, "s-s-s": 5, "fp8": 6}
N_MLP_PARAMS = 4866


class GadiError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__(f"{what}: {status_str(status)} ({status})")


class _Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("val", ctypes.c_void_p), ("on_device", ctypes.c_int32)]


class _Options(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int), ("eps_inner", ctypes.c_double), ("maxit_outer", ctypes.c_int32),
                ("maxit_inner", ctypes.c_int32), ("on_device", ctypes.c_int32),
                ("record_history", ctypes.c_int32), ("prune_dominated", ctypes.c_int32),
                ("grid_per_system", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("outer_sweeps", ctypes.c_int32), ("inner_H", ctypes.c_int64),
                ("inner_S", ctypes.c_int64), ("relres", ctypes.c_double), ("seconds", ctypes.c_double),
                ("alpha", ctypes.c_double), ("omega", ctypes.c_double), ("fell_back", ctypes.c_int32),
                ("barriers", ctypes.c_int64), ("barrier_seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _load():
    path = _build.ensure_built()
    # One HIP runtime per process: torch ships its own libamdhip64.so.7 and
    # loads it by path.  Loaded first, it also satisfies libgadi's dependency
    # of that name; loaded after libgadi, it would be a second runtime beside
    # the system one, and whichever initialises second finds no device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    sigs = {
        "gadi_setup": (i32, [P(_Csr), ctypes.c_int, P(vp)]),
        "gadi_set_stream": (i32, [vp, vp]),
        "gadi_ir_solve": (i32, [vp, vp, vp, f64, f64, f64, P(_Options), P(SolveInfo)]),
        "gadi_ir_solve_noalloc": (i32, [vp, vp, vp, f64, f64, f64, P(_Options), P(SolveInfo)]),
        "gadi_get_history": (i32, [vp, P(f64), i32]),
        "gadi_ir_solve_batched": (i32, [P(vp), i32, P(vp), P(vp), P(f64), P(f64), i32, f64, P(_Options),
                                        P(SolveInfo)]),
        "gadi_spmv": (i32, [vp, i32, f64, vp, vp]),
        "gadi_get_split_fp16": (i32, [vp, i32, vp, vp, vp, P(i64)]),
        "gadi_get_split_fp8": (i32, [vp, i32, vp, vp, vp, P(i64)]),
        "gadi_get_layout": (i32, [vp, P(i64)]),
        "gadi_get_phase_profile": (i32, [vp, P(f64), P(i64)]),
        "gadi_get_block_profile": (i32, [vp, P(f64), P(f64), i32]),
        "gadi_get_phase_block_profile": (i32, [vp, P(f64), P(i32), i32]),
        "gadi_features": (i32, [vp, i32, i32, P(f64), P(ctypes.c_float)]),
        "gadi_mlp_create": (i32, [ctypes.c_uint64, P(vp)]),
        "gadi_mlp_destroy": (i32, [vp]),
        "gadi_mlp_set_weights": (i32, [vp, vp]),
        "gadi_mlp_get_weights": (i32, [vp, vp]),
        "gadi_mlp_set_norm": (i32, [vp, vp, vp]),
        "gadi_mlp_get_norm": (i32, [vp, vp, vp]),
        "gadi_mlp_set_bounds": (i32, [vp, vp, vp]),
        "gadi_mlp_get_bounds": (i32, [vp, vp, vp]),
        "gadi_mlp_forward": (i32, [vp, vp, i32, vp]),
        "gadi_mlp_loss_grad": (i32, [vp, vp, vp, i32, vp, vp]),
        "gadi_train_mlp": (i32, [vp, vp, vp, i32, i32, ctypes.c_float, vp]),
        "gadi_predict_params": (i32, [vp, vp, P(f64), P(f64)]),
        "gadi_destroy": (i32, [vp]),
        "gadi_status_str": (ctypes.c_char_p, [i32]),
        "gadi_solver_blocks": (i32, [vp, P(i32)]),
        "gadi_solver_form": (i32, [vp]),
        "gadi_default_options": (None, [P(_Options), ctypes.c_int]),
        "gadi_sylv_setup": (i32, [i32, i32, vp, vp, vp, vp, vp, vp, P(vp)]),
        "gadi_sylv_solve": (i32, [vp, vp, vp, f64, f64, f64, P(_Options), P(SolveInfo)]),
        "gadi_sylv_get_history": (i32, [vp, P(f64), i32]),
        "gadi_sylv_set_stream": (i32, [vp, vp]),
        "gadi_sylv_destroy": (i32, [vp]),
        "gadi_gpr_fit": (i32, [P(f64), P(f64), i32, P(vp)]),
        "gadi_gpr_predict": (i32, [vp, P(f64), i32, P(f64), P(f64)]),
        "gadi_gpr_params": (i32, [vp, P(f64)]),
        "gadi_gpr_destroy": (i32, [vp]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()

# Handles that still own library memory.  They are destroyed by an exit hook
# that runs before module teardown and before the HIP runtime's own shutdown,
# so no device buffer, event or handle outlives the runtime (a profiler that
# finalises at exit then sees every allocation released).
_live = weakref.WeakSet()


def _track(obj):
    _live.add(obj)


@atexit.register
def _close_all():
    for obj in list(_live):
        try:
            obj.close()
        except Exception:  # pragma: no cover - exit path, nothing to report to
            pass


def lib():
    return _lib


def status_str(s: int) -> str:
    return _lib.gadi_status_str(int(s)).decode()


def _check(st, what):
    if st != OK:
        raise GadiError(st, what)


def _is_device_tensor(a) -> bool:
    try:
        import torch
        return isinstance(a, torch.Tensor) and a.is_cuda
    except ImportError:  # pragma: no cover
        return False


def _current_stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def options(prec="fp16", eps_inner=None, maxit_outer=20000, maxit_inner=2000, on_device=False, history=False):
    o = _Options()
    _lib.gadi_default_options(ctypes.byref(o), PREC[prec])
    if eps_inner is not None:
        o.eps_inner = float(eps_inner)
    o.maxit_outer = int(maxit_outer)
    o.maxit_inner = int(maxit_inner)
    o.on_device = 1 if on_device else 0
    o.record_history = 1 if history else 0
    return o


class System:
    """A sparse system prepared on the device: A, its HSS splitting, solver workspace.

    `A` is any object with n, row_ptr (int32), col (int32), val (float64)
    numpy arrays, e.g. gadi_inputs.Csr.
    """

    def __init__(self, A):
        self.n = int(A.n)
        rp = np.ascontiguousarray(A.row_ptr, dtype=np.int32)
        col = np.ascontiguousarray(A.col, dtype=np.int32)
        val = np.ascontiguousarray(A.val, dtype=np.float64)
        c = _Csr(self.n, int(rp[-1]), rp.ctypes.data, col.ctypes.data, val.ctypes.data, 0)
        h = ctypes.c_void_p()
        _check(_lib.gadi_setup(ctypes.byref(c), 0, ctypes.byref(h)), "gadi_setup")
        self._h = h
        self.meta = A
        self.history = None
        _track(self)

    def close(self):
        # at interpreter exit the module globals may already be gone: nothing to free then
        if getattr(self, "_h", None) and _lib is not None:
            _lib.gadi_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    @property
    def handle(self):
        return self._h

    def bind_current_stream(self):
        _check(_lib.gadi_set_stream(self._h, _current_stream()), "gadi_set_stream")

    def solve(self, b, alpha=0.5, omega=0.5, tol=1e-10, x0=None, prec="fp16", eps_inner=None,
              maxit_outer=20000, maxit_inner=2000, history=False, check=False):
        """GADI-IR solve.  b (and x0) as numpy float64 (host) or torch float64 CUDA tensors.

        Returns (x, info-dict).  With check=True a non-OK status raises."""
        dev = _is_device_tensor(b)
        if dev:
            import torch
            self.bind_current_stream()
            x = torch.zeros_like(b) if x0 is None else x0.clone()
            bp, xp = b.data_ptr(), x.data_ptr()
        else:
            b = np.ascontiguousarray(b, dtype=np.float64)
            x = np.zeros(self.n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
            bp, xp = b.ctypes.data, x.ctypes.data
        if len(b) != self.n:
            raise ValueError("b has the wrong length")
        o = options(prec, eps_inner, maxit_outer, maxit_inner, dev, history)
        info = SolveInfo()
        st = _lib.gadi_ir_solve(self._h, ctypes.c_void_p(bp), ctypes.c_void_p(xp), float(alpha), float(omega),
                                float(tol), ctypes.byref(o), ctypes.byref(info))
        if check:
            _check(st, "gadi_ir_solve")
        if history and st in (OK, EMAXIT, EDIVERGED):
            buf = np.zeros(maxit_outer + 1)
            k = _lib.gadi_get_history(self._h, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(buf))
            self.history = buf[:k]
        elif history:
            self.history = np.zeros(0)
        d = info.as_dict()
        d["status_str"] = status_str(st)
        return x, d

    def solve_noalloc(self, b, x, alpha=0.5, omega=0.5, tol=1e-10, prec="fp16", eps_inner=None,
                      maxit_outer=20000, maxit_inner=2000):
        """gadi_ir_solve_noalloc: the solve with the library's fixed scratch array as
        workspace (no device allocation).  b, x: float64 CUDA tensors of length n; x
        is the start and receives the result.  Returns the info dict."""
        if not (_is_device_tensor(b) and _is_device_tensor(x)):
            raise ValueError("solve_noalloc takes device tensors")
        if len(b) != self.n or len(x) != self.n:
            raise ValueError("b and x must have length n")
        self.bind_current_stream()
        o = options(prec, eps_inner, maxit_outer, maxit_inner, True, False)
        info = SolveInfo()
        st = _lib.gadi_ir_solve_noalloc(self._h, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                        float(alpha), float(omega), float(tol), ctypes.byref(o), ctypes.byref(info))
        d = info.as_dict()
        d["status"] = st
        d["status_str"] = status_str(st)
        return d

    def spmv(self, which: str, x, y, alpha=1.0):
        """Device product on torch tensors: which in {'A','H16','S16','H64','H8'}."""
        code = {"A": 0, "H16": 1, "S16": 2, "H64": 3, "H8": 4}[which]
        self.bind_current_stream()
        _check(_lib.gadi_spmv(self._h, code, float(alpha), ctypes.c_void_p(x.data_ptr()),
                              ctypes.c_void_p(y.data_ptr())), "gadi_spmv")

    def split_fp16(self, which: str):
        """The packed fp16 values of 'H' or 'S' in CSR order of the union pattern (with diagonal)."""
        code = {"H": 1, "S": 2}[which]
        nnz = ctypes.c_int64(0)
        _check(_lib.gadi_get_split_fp16(self._h, code, None, None, None, ctypes.byref(nnz)), "split")
        rp = np.empty(self.n + 1, np.int32)
        col = np.empty(nnz.value, np.int32)
        val = np.empty(nnz.value, np.uint16)
        _check(_lib.gadi_get_split_fp16(self._h, code, ctypes.c_void_p(rp.ctypes.data),
                                        ctypes.c_void_p(col.ctypes.data), ctypes.c_void_p(val.ctypes.data),
                                        ctypes.byref(nnz)), "split")
        return rp, col, val.view(np.float16)

    def split_fp8(self, which: str):
        """E4M3 codes of the off-diagonal values of 'H' or 'S' in CSR order of the union pattern."""
        code = {"H": 1, "S": 2}[which]
        nnz = ctypes.c_int64(0)
        _check(_lib.gadi_get_split_fp8(self._h, code, None, None, None, ctypes.byref(nnz)), "split")
        rp = np.empty(self.n + 1, np.int32)
        col = np.empty(nnz.value, np.int32)
        val = np.empty(nnz.value, np.uint8)
        _check(_lib.gadi_get_split_fp8(self._h, code, ctypes.c_void_p(rp.ctypes.data),
                                       ctypes.c_void_p(col.ctypes.data), ctypes.c_void_p(val.ctypes.data),
                                       ctypes.byref(nnz)), "split")
        return rp, col, val

    PHASES = ("residual", "cg_start", "cg_product", "cg_update", "cgne_start", "cgne_product1",
              "cgne_product2", "cgne_update", "x_update")

    def phase_profile(self):
        """Block 0's compute seconds and counts per phase of the last solve."""
        sec = (ctypes.c_double * 10)()
        cnt = (ctypes.c_int64 * 10)()
        _check(_lib.gadi_get_phase_profile(self._h, sec, cnt), "gadi_get_phase_profile")
        return {k: (sec[i], cnt[i]) for i, k in enumerate(self.PHASES)}

    def block_profile(self):
        """(seconds inside barriers, seconds in the launch) per block of the last solve launch."""
        w = np.zeros(4096)
        t = np.zeros(4096)
        k = _lib.gadi_get_block_profile(self._h, w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 4096)
        return w[:k], t[:k]

    def phase_block_profile(self, max_phases=96):
        """(seconds [phases, blocks], phase ids [phases]) of the first phases of the last solve launch."""
        nb, _ = self.solver_blocks()
        sec = np.zeros(max_phases * max(nb, 1))
        ids = np.zeros(max_phases, np.int32)
        k = _lib.gadi_get_phase_block_profile(self._h, sec.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                              ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), max_phases)
        return sec[:k * nb].reshape(k, nb), ids[:k]

    def layout(self):
        """Packed layout counts: dict with n, npad, nnz_off, slots, dia_slots,
        explicit_entries, uniform_offsets (offsets per slice of a uniformly
        diagonal-style layout, 0 if per-slice metadata is used)."""
        out = (ctypes.c_int64 * 7)()
        _check(_lib.gadi_get_layout(self._h, out), "gadi_get_layout")
        return dict(zip(("n", "npad", "nnz_off", "slots", "dia_slots", "explicit_entries", "uniform_offsets"),
                        list(out)))

    def features(self, dim, grid, beta):
        beta = np.ascontiguousarray(np.broadcast_to(np.asarray(beta, dtype=np.float64), (dim,)))
        out = np.zeros(8, np.float32)
        _check(_lib.gadi_features(self._h, int(dim), int(grid),
                                  beta.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))), "gadi_features")
        return out

    def solver_blocks(self):
        """(blocks, threads per block) of the last solve launch."""
        t = ctypes.c_int32(0)
        nb = _lib.gadi_solver_blocks(self._h, ctypes.byref(t))
        return int(nb), int(t.value)

    def solver_form(self):
        """Inner-solver form of the last solve launch (0 Hestenes-Stiefel,
        1 Chronopoulos-Gear, 2 pipelined CG with Craig's CGNE, 3 Hestenes-Stiefel
        CG with Craig's CGNE; -1 before any)."""
        return int(_lib.gadi_solver_form(self._h))


def solve_batched(systems, bs, alphas, omegas, tol=1e-10, prec="fp16", eps_inner=None, maxit_outer=5000,
                  maxit_inner=2000, want_x=False, prune=False):
    """Batched (alpha, omega) sweep over many systems in one persistent launch.

    systems: list of System; bs: list of numpy float64 right-hand sides;
    alphas, omegas: the trial grid, either one list for every system (<= 16
    trials) or one list per system (nested, same length).
    Returns (records [nsys][ntrial] dicts, xs or None)."""
    per_sys = np.ndim(alphas) == 2
    nsys = len(systems)
    nt = len(alphas[0]) if per_sys else len(alphas)
    hs = (ctypes.c_void_p * nsys)(*[s.handle.value for s in systems])
    bsa = [np.ascontiguousarray(b, dtype=np.float64) for b in bs]
    bp = (ctypes.c_void_p * nsys)(*[b.ctypes.data for b in bsa])
    xs = [np.zeros(s.n) for s in systems] if want_x else None
    xp = (ctypes.c_void_p * nsys)(*([x.ctypes.data for x in xs] if want_x else [None] * nsys))
    al = np.ascontiguousarray(np.asarray(alphas, dtype=np.float64).ravel())
    om = np.ascontiguousarray(np.asarray(omegas, dtype=np.float64).ravel())
    o = options(prec, eps_inner, maxit_outer, maxit_inner, False, False)
    o.prune_dominated = 1 if prune else 0
    o.grid_per_system = 1 if per_sys else 0
    infos = (SolveInfo * (nsys * nt))()
    st = _lib.gadi_ir_solve_batched(hs, nsys, bp, xp, al.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    om.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), nt, float(tol),
                                    ctypes.byref(o), infos)
    if st not in (OK, EMAXIT):
        _check(st, "gadi_ir_solve_batched")
    recs = [[infos[s * nt + t].as_dict() for t in range(nt)] for s in range(nsys)]
    return recs, xs


class Predictor:
    """(alpha, omega) predictor: the 8 -> 64 -> 64 -> 2 MLP with device kernels."""

    def __init__(self, seed=0):
        h = ctypes.c_void_p()
        _check(_lib.gadi_mlp_create(int(seed), ctypes.byref(h)), "gadi_mlp_create")
        self._h = h
        _track(self)

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.gadi_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def set_weights(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        assert w.size == N_MLP_PARAMS
        _check(_lib.gadi_mlp_set_weights(self._h, ctypes.c_void_p(w.ctypes.data)), "set_weights")

    def weights(self):
        w = np.zeros(N_MLP_PARAMS, np.float32)
        _check(_lib.gadi_mlp_get_weights(self._h, ctypes.c_void_p(w.ctypes.data)), "get_weights")
        return w

    def set_norm(self, mu, sd):
        mu = np.ascontiguousarray(mu, dtype=np.float32)
        sd = np.ascontiguousarray(sd, dtype=np.float32)
        _check(_lib.gadi_mlp_set_norm(self._h, ctypes.c_void_p(mu.ctypes.data), ctypes.c_void_p(sd.ctypes.data)),
               "set_norm")

    def norm(self):
        """(mu, sd) feature standardisation in use."""
        mu = np.zeros(8, np.float32)
        sd = np.zeros(8, np.float32)
        _check(_lib.gadi_mlp_get_norm(self._h, ctypes.c_void_p(mu.ctypes.data), ctypes.c_void_p(sd.ctypes.data)),
               "get_norm")
        return mu, sd

    def set_bounds(self, lo, hi):
        lo = np.ascontiguousarray(lo, dtype=np.float32)
        hi = np.ascontiguousarray(hi, dtype=np.float32)
        _check(_lib.gadi_mlp_set_bounds(self._h, ctypes.c_void_p(lo.ctypes.data), ctypes.c_void_p(hi.ctypes.data)),
               "set_bounds")

    def bounds(self):
        lo = np.zeros(8, np.float32)
        hi = np.zeros(8, np.float32)
        _check(_lib.gadi_mlp_get_bounds(self._h, ctypes.c_void_p(lo.ctypes.data), ctypes.c_void_p(hi.ctypes.data)),
               "get_bounds")
        return lo, hi

    def forward(self, X):
        X = np.ascontiguousarray(X, dtype=np.float32)
        Y = np.zeros((X.shape[0], 2), np.float32)
        _check(_lib.gadi_mlp_forward(self._h, ctypes.c_void_p(X.ctypes.data), X.shape[0],
                                     ctypes.c_void_p(Y.ctypes.data)), "forward")
        return Y

    def loss_grad(self, Xs, Y):
        Xs = np.ascontiguousarray(Xs, dtype=np.float32)
        Y = np.ascontiguousarray(Y, dtype=np.float32)
        g = np.zeros(N_MLP_PARAMS, np.float32)
        L = np.zeros(1, np.float32)
        _check(_lib.gadi_mlp_loss_grad(self._h, ctypes.c_void_p(Xs.ctypes.data), ctypes.c_void_p(Y.ctypes.data),
                                       Xs.shape[0], ctypes.c_void_p(L.ctypes.data), ctypes.c_void_p(g.ctypes.data)),
               "loss_grad")
        return float(L[0]), g

    def train(self, X, Y, epochs=2000, lr=3e-3):
        X = np.ascontiguousarray(X, dtype=np.float32)
        Y = np.ascontiguousarray(Y, dtype=np.float32)
        losses = np.zeros(epochs, np.float32)
        _check(_lib.gadi_train_mlp(self._h, ctypes.c_void_p(X.ctypes.data), ctypes.c_void_p(Y.ctypes.data),
                                   X.shape[0], int(epochs), float(lr), ctypes.c_void_p(losses.ctypes.data)),
               "gadi_train_mlp")
        return losses

    def predict(self, features):
        f = np.ascontiguousarray(features, dtype=np.float32)
        a, w = ctypes.c_double(), ctypes.c_double()
        _check(_lib.gadi_predict_params(self._h, ctypes.c_void_p(f.ctypes.data), ctypes.byref(a), ctypes.byref(w)),
               "gadi_predict_params")
        return a.value, w.value


class Sylvester:
    """GADI-AB for the continuous Sylvester equation A X + X B = C (libgadi's
    gadi_sylv_*).  A (m x m) and B (n x n) are tridiagonal triples
    (sub[k-1], diag[k], sup[k-1]) of float64 arrays, T[i+1, i] = sub[i]."""

    def __init__(self, A, B):
        a = [np.ascontiguousarray(v, dtype=np.float64) for v in A]
        b = [np.ascontiguousarray(v, dtype=np.float64) for v in B]
        self.m, self.n = len(a[1]), len(b[1])
        h = ctypes.c_void_p()
        ptr = lambda v: ctypes.c_void_p(v.ctypes.data) if v.size else None
        _check(_lib.gadi_sylv_setup(self.m, self.n, ptr(a[0]), ptr(a[1]), ptr(a[2]), ptr(b[0]), ptr(b[1]), ptr(b[2]),
                                    ctypes.byref(h)), "gadi_sylv_setup")
        self._h = h
        self.history = np.zeros(0)
        _track(self)

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.gadi_sylv_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def solve(self, C, alpha=0.5, omega=0.5, tol=1e-10, x0=None, prec="fp16", maxit_outer=20000, history=False):
        """C (and x0) as (m, n) numpy float64 (host) or torch float64 CUDA tensors.
        prec in {'fp64', 'fp32', 'fp16'}.  Returns (X, info-dict)."""
        if prec not in ("fp64", "fp32", "fp16"):
            raise ValueError("GADI-AB runs its inner solves in fp64, fp32 or fp16")
        dev = _is_device_tensor(C)
        if dev:
            import torch
            _check(_lib.gadi_sylv_set_stream(self._h, _current_stream()), "gadi_sylv_set_stream")
            C = C.contiguous()
            X = torch.zeros_like(C) if x0 is None else x0.clone().contiguous()
            cp, xp = C.data_ptr(), X.data_ptr()
        else:
            _check(_lib.gadi_sylv_set_stream(self._h, None), "gadi_sylv_set_stream")
            C = np.ascontiguousarray(C, dtype=np.float64)
            X = np.zeros_like(C) if x0 is None else np.array(x0, dtype=np.float64, copy=True, order="C")
            cp, xp = C.ctypes.data, X.ctypes.data
        if tuple(C.shape) != (self.m, self.n) or tuple(X.shape) != (self.m, self.n):
            raise ValueError("C and x0 must be m x n")
        o = options(prec, None, maxit_outer, 1, dev, history)
        info = SolveInfo()
        st = _lib.gadi_sylv_solve(self._h, ctypes.c_void_p(cp), ctypes.c_void_p(xp), float(alpha), float(omega),
                                  float(tol), ctypes.byref(o), ctypes.byref(info))
        if st not in (OK, EMAXIT, EDIVERGED, EOVERFLOW16):
            _check(st, "gadi_sylv_solve")
        if history:
            buf = np.zeros(maxit_outer + 1)
            k = _lib.gadi_sylv_get_history(self._h, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(buf))
            self.history = buf[:k]
        d = info.as_dict()
        d["status_str"] = status_str(st)
        return X, d
