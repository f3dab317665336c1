"""Build libarkcos.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1211_3556_amd.build [--force]

Every HIP source is compiled for gfx950 only.  Packed FP32 instructions are
disabled (-packed-fp32-ops): ordinary scalar float code is vectorised by the
compiler otherwise.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libarkcos.so")
SOURCES = ["plan.hip", "kernels.hip", "capi.hip", "sht.hip", "tune.hip", "rotate.hip"]
HEADERS = [os.path.join(CSRC, "arkcos_internal.hpp"), os.path.join(INCLUDE, "arkcos.h")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ROCM_LIB = "/opt/rocm/lib"   # roctx (profiler ranges around the entry points)
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH, "-Wall", "-Wno-unused-function",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-munsafe-fp-atomics", "-I", INCLUDE, "-I", CSRC]


def _obj(src: str) -> str:
    return os.path.join(CSRC, os.path.splitext(src)[0] + ".o")


def _compile(src: str) -> None:
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", _obj(src)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr))
    # the host pass warns that it does not know the packed-FP32 feature; drop that line
    noise = "packed-fp32-ops"
    for line in r.stderr.splitlines():
        if noise not in line and line.strip() and "warning generated" not in line:
            sys.stderr.write(line + "\n")


def build(force: bool = True) -> str:
    """Compile every HIP source for gfx950 and link libarkcos.so."""
    stale = force or not os.path.exists(LIB)
    if not stale:
        t = os.path.getmtime(LIB)
        stale = any(os.path.getmtime(os.path.join(CSRC, s)) > t for s in SOURCES) or \
            any(os.path.getmtime(h) > t for h in HEADERS)
    if not stale:
        return LIB
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, *[_obj(s) for s in SOURCES],
           "-L" + ROCM_LIB, "-lrocprofiler-sdk-roctx", "-Wl,-rpath," + ROCM_LIB, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, LIB)
    for s in SOURCES:
        try:
            os.remove(_obj(s))
        except OSError:
            pass
    return LIB


if __name__ == "__main__":
    print(build(force="--force" in sys.argv or True))
