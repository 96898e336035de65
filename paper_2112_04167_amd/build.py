"""Build the HIP library (gfx950) in-tree: paper_2112_04167_amd/_lib/libdgsipdg.so.

Every HIP source is compiled by hipcc for gfx950 only, with packed-FP32
instructions disabled, then linked into one shared library that exports the
C-ABI of include/dg_sipdg.h.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_lib")
OBJ = os.path.join(OUT, "obj")
LIB = os.path.join(OUT, "libdgsipdg.so")
SOURCES = ["gll_host.cpp", "kernels.hip", "cg_kernels.hip", "solver.cpp", "batched.hip", "server.cpp",
           "fdm_host.cpp", "fdm.hip", "projection.hip", "convection.hip", "imex.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-Wall", "-Wno-unused-function",
         "-Wno-unused-variable"]


def _compile(src):
    path = os.path.join(CSRC, src)
    obj = os.path.join(OBJ, src + ".o")
    cmd = [HIPCC] + FLAGS + ["-x", "hip", "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    return src, r.returncode, r.stdout + r.stderr, obj


def build(verbose=True, jobs=None):
    os.makedirs(OBJ, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 4)))
    objs = []
    failed = False
    with cf.ThreadPoolExecutor(jobs) as ex:
        for src, rc, out, obj in ex.map(_compile, srcs):
            warn = [l for l in out.splitlines() if "packed-fp32-ops" not in l and l.strip()]
            if rc != 0:
                failed = True
                print("=== %s FAILED\n%s" % (src, out), file=sys.stderr)
            elif verbose and warn:
                print("=== %s\n%s" % (src, "\n".join(warn[:40])))
            objs.append(obj)
    if failed:
        raise RuntimeError("HIP build failed")
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread", "-lrocprofiler-sdk-roctx"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build()
