"""Host sanitizer checks: the library's host code (argument checks, workspace
sizing and planning of the C ABI) and the oracle, built with AddressSanitizer
and UndefinedBehaviorSanitizer (clang, device code untouched), run the C-ABI
contract tests and a set of oracle pins in a child process with the clang ASan
runtime preloaded; any report ends the child with a failure."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "_build_asan")
RT = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))

PINS = ("two_point or hamiltonian or closed_forms or integer_coord or brute_force_cells or "
        "reduces_to_exact or coincident or bh_matches_bruteforce or exact_rows or other_points "
        "or adjoint_matches_autograd or bh_adjoint_limits")

CHECK_LOADED = r"""
import sys
sys.path.insert(0, {root!r})
from paper_1907_04834_amd import gs
from oracle import oracle as O
gs.lib(); O.lib()
maps = open("/proc/self/maps").read()
assert "libclang_rt.asan" in maps, "ASan runtime not loaded"
assert "libgsbh_asan.so" in maps and "liboracle_asan.so" in maps, "sanitized builds not loaded"
print("sanitized builds loaded")
"""


@pytest.mark.skipif(not RT, reason="clang ASan runtime not found")
def test_host_code_under_address_and_ub_sanitizers():
    from oracle import oracle as O
    from paper_1907_04834_amd import build

    lib = build.build_sanitized(OUT)
    olib = O.build_sanitized(os.path.join(OUT, "liboracle_asan.so"))
    env = dict(os.environ, LD_PRELOAD=RT[-1], GSBH_LIB=lib, GS_ORACLE_LIB=olib,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    run = dict(env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    r = subprocess.run([sys.executable, "-c", CHECK_LOADED.format(root=ROOT)], **run)
    assert r.returncode == 0, r.stdout + r.stderr
    for args in (["tests/test_capi_cpu.py"], ["tests/test_oracle_pins.py", "-k", PINS]):
        r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                            *args], **run)
        assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
