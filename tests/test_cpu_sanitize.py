"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The C oracle (setup and splitting, products, GADI, Gershgorin bounds) and the
host-only GPR of libgadi (`csrc/gpr.cpp`) are compiled with gcc/g++ and
-fsanitize=address,undefined into a small driver (`tests/sanitize/host_driver.cpp`),
which runs them on a 2-D convection-diffusion system and a GPR fit; any memory
or undefined-behaviour error aborts the driver.  The device code cannot run
under a sanitizer here (no GPU, and GPU sanitizers are not used), so the host
parts are what this covers.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


@pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None, reason="no host compiler")
def test_host_code_under_sanitizers(tmp_path):
    obj_oracle = str(tmp_path / "oracle.o")
    exe = str(tmp_path / "host_driver")
    subprocess.run(["gcc", "-std=c11", "-fopenmp", "-ffp-contract=off", "-c", *SAN,
                    os.path.join(ROOT, "oracle", "gadi_oracle.c"), "-o", obj_oracle],
                   check=True, capture_output=True)
    subprocess.run(["g++", "-std=c++17", "-fopenmp", *SAN, "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"),
                    os.path.join(ROOT, "paper_2501_04229_amd", "csrc", "gpr.cpp"), obj_oracle, "-o", exe],
                   check=True, capture_output=True)
    # verify_asan_link_order=0: a library the environment preloads may precede the ASan runtime
    env = dict(os.environ, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
    assert "host driver ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
