"""CPU-side checks of the C ABI: the library loads and exports what include/gadi.h declares."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gadi.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(gadi_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("gadi_setup", "gadi_ir_solve", "gadi_ir_solve_batched", "gadi_predict_params",
                 "gadi_features", "gadi_train_mlp", "gadi_destroy", "gadi_status_str"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2501_04229_amd as gadi
    lib = ctypes.CDLL(gadi.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", gadi.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (gadi_[a-z0-9_]+)", out))
    assert set(_declared()) <= exported


def test_status_strings_and_defaults():
    import paper_2501_04229_amd as gadi
    assert gadi.status_str(0) == "ok"
    assert gadi.status_str(4) == "diverged"
    assert gadi.status_str(gadi.EPRUNED).startswith("pruned")
    assert gadi.status_str(99) == "unknown status"
    o = gadi.options("fp64")
    assert o.prec == 0 and o.eps_inner == 1e-6
    o = gadi.options("fp16")
    assert o.prec == 1 and 0 < o.eps_inner < 1


def test_library_is_built_for_gfx950():
    import paper_2501_04229_amd as gadi
    data = open(gadi.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_argument_checks_without_gpu():
    """Null handles and bad enums are rejected before any device call."""
    import paper_2501_04229_amd as gadi
    L = gadi.lib()
    h = ctypes.c_void_p()
    assert L.gadi_setup(None, 0, ctypes.byref(h)) == gadi.EINVAL
    assert L.gadi_ir_solve(None, None, None, 0.5, 0.5, 1e-10, None, None) == gadi.EINVAL
    assert L.gadi_destroy(None) == gadi.EINVAL
    assert L.gadi_spmv(None, 0, 1.0, None, None) == gadi.EINVAL


def test_one_hip_runtime_when_the_package_is_imported_first():
    """Imported before torch (as `python -m paper_2501_04229_amd.<module>` does),
    the package must still leave one libamdhip64 in the process: a second
    runtime beside torch's finds no device."""
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import paper_2501_04229_amd, torch\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "print(len({l.split()[-1] for l in maps if 'libamdhip64' in l}))\n") % ROOT
    out = subprocess.run([os.sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    assert out.stdout.strip().splitlines()[-1] == "1"


def test_live_handles_are_closed_by_the_exit_hook():
    """Every handle that owns library memory is registered, and the exit hook closes it
    (host-only GPR handle: no device needed)."""
    import numpy as np
    import paper_2501_04229_amd as gadi
    from paper_2501_04229_amd.predictor.gpr import GPR
    g = GPR(np.array([1.0, 2.0, 3.0, 4.0]), np.array([0.5, 0.1, -0.2, -0.6]))
    assert g in gadi._live and g._h
    gadi._close_all()
    assert g._h is None
