"""Build libwd.so (gfx950) with hipcc, in-tree.

The line-tile passes are compiled once per value type and tile variant
(points per thread 1, 2, 4, 8) from wd_line.hip; every translation unit is
compiled in parallel and the objects are linked into one shared library.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libwd.so")
ARCH = os.environ.get("WD_OFFLOAD_ARCH", "gfx950")

FLAGS = ["hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
         # keep the compiler from emitting packed FP32 instructions
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result", "-Wno-unused-function",
         "-I", os.path.join(ROOT, "include"), "-I", HERE]


def _units():
    """(source, extra flags, object name) of every translation unit."""
    out = [("wd_kernels.hip", [], "wd_kernels.o"),
           ("wd_seg.hip", [], "wd_seg.o"),
           ("wd_host.cpp", [], "wd_host.o"),
           ("wd_server.cpp", [], "wd_server.o")]
    for t, tag in (("float", "f32"), ("double", "f64")):
        for np_ in (1, 2, 4, 8):
            fn = f"line_launch_{tag}_{np_}"
            out.append(("wd_line.hip",
                        [f"-DWD_LINE_T={t}", f"-DWD_LINE_NP={np_}", f"-DWD_LINE_FN={fn}"],
                        f"wd_line_{tag}_{np_}.o"))
    return out


def build(verbose: bool = False, jobs: int = 0) -> str:
    jobs = jobs or min(8, os.cpu_count() or 1)
    tmpdir = tempfile.mkdtemp(prefix="wd_build_")
    try:
        def compile_one(u):
            src, extra, obj = u
            cmd = FLAGS + extra + ["-c", os.path.join(HERE, src), "-o", os.path.join(tmpdir, obj)]
            if verbose:
                print(" ".join(cmd), flush=True)
            r = subprocess.run(cmd, capture_output=True, text=True)
            return obj, r.returncode, r.stderr

        with ThreadPoolExecutor(max_workers=jobs) as ex:
            results = list(ex.map(compile_one, _units()))
        failed = [(o, e) for o, rc, e in results if rc != 0]
        for o, rc, e in results:
            if e.strip() and (verbose or rc != 0):
                print(f"--- {o}\n{e}", file=sys.stderr, flush=True)
        if failed:
            raise RuntimeError("libwd build failed: " + ", ".join(o for o, _ in failed))
        tmp = LIB + ".tmp"
        link = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + \
               [os.path.join(tmpdir, o) for _, _, o in _units()] + ["-lpthread"]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.check_call(link)
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
