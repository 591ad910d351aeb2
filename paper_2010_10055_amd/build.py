"""Build the HIP library (libdibella.so) for gfx950 with hipcc, in tree, and
beside it the benchmark's counter-calibration kernels (libdibella_calib.so),
which the library does not contain."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libdibella.so")
SOURCES = ["runtime.hip", "overlap.hip", "tr.hip", "rseeds.hip", "noalloc.hip", "kmer.hip", "align.hip", "api.hip"]
CALIB_SOURCE = "calib.hip"
CALIB_OUT = os.path.join(HERE, "libdibella_calib.so")
ARCH = os.environ.get("DIBELLA_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I" + os.path.join(ROOT, "include"),
         "-Wall", "-Wno-unused-function",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src: str, objdir: str) -> str:
    obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
    cmd = ["hipcc", *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{msg}")
    if msg.strip():
        print(msg, file=sys.stderr)
    return obj


def _link(objs, out: str) -> None:
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, out)


def build(verbose: bool = True) -> str:
    objdir = os.path.join(ROOT, "_build")
    os.makedirs(objdir, exist_ok=True)
    srcs = SOURCES + [CALIB_SOURCE]
    with ThreadPoolExecutor(max_workers=len(srcs)) as ex:
        objs = list(ex.map(lambda s: _compile(s, objdir), srcs))
    _link(objs[:len(SOURCES)], OUT)
    _link(objs[len(SOURCES):], CALIB_OUT)
    if verbose:
        print("built", OUT, "and", os.path.basename(CALIB_OUT))
    return OUT


if __name__ == "__main__":
    build()
