"""Build libgsbh.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1907_04834_amd.build [--jobs N]

Every source under csrc/ is compiled to an object under _build/ and linked
into paper_1907_04834_amd/libgsbh.so.  Packed FP32 instructions are disabled
for the device code (-packed-fp32-ops).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libgsbh.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wall", "-Wno-unused-function",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) +
                  glob.glob(os.path.join(CSRC, "*.cpp")))


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, "-x", "hip", *FLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    if r.stderr.strip():
        # warnings other than the host pass not knowing the packed-fp32 feature
        lines = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln]
        if any(ln.strip() for ln in lines):
            sys.stderr.write("\n".join(lines) + "\n")
    return obj


def ensure_built() -> str:
    """Builds the library only when it is missing (tests, smoke and the
    benchmark use what is built; the binding itself never builds)."""
    return LIB if os.path.exists(LIB) else build()


def build(jobs: int = 8) -> str:
    """Compile every source and link the shared library; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=max(1, min(jobs, 16))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def build_sanitized(out_dir: str, jobs: int = 8) -> str:
    """The library with its host code built with AddressSanitizer and
    UndefinedBehaviorSanitizer (device code as usual), into out_dir; for the
    sanitizer checks of the test suite, which load it with the clang ASan
    runtime preloaded.  Returns the library path."""
    global BUILD, LIB, FLAGS
    saved = (BUILD, LIB, FLAGS)
    try:
        BUILD = out_dir
        LIB = os.path.join(out_dir, "libgsbh_asan.so")
        FLAGS = FLAGS + SAN_FLAGS
        os.makedirs(BUILD, exist_ok=True)
        with cf.ThreadPoolExecutor(max_workers=max(1, min(jobs, 16))) as ex:
            objs = list(ex.map(_compile, sources()))
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-shared-libasan", *SAN_FLAGS,
               "-o", LIB, *objs]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed:\n{r.stderr}")
        return LIB
    finally:
        BUILD, LIB, FLAGS = saved


def asm(src_name: str, out: str) -> None:
    """Write the gfx950 assembly of one source (for inspection)."""
    src = os.path.join(CSRC, src_name)
    cmd = [HIPCC, "-x", "hip", *FLAGS, "--cuda-device-only", "-S", src, "-o", out]
    subprocess.run(cmd, check=True)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("--asm", default=None, help="source file name to dump as assembly")
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    if a.asm:
        asm(a.asm, a.out or os.path.join(BUILD, a.asm + ".s"))
    else:
        print(build(a.jobs))
