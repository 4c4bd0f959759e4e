"""Build liblsms_kkr.so (HIP for gfx950 + host C++) in place, with hipcc.

Usage: python -m paper_2311_12134_amd.build   (or build() from Python)
"""

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "liblsms_kkr.so")
OBJ = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

DEVICE_SOURCES = ["assemble.hip", "lu.hip", "gemm.hip", "gemm64.hip", "gemm_persist.hip", "gemm_wide.hip", "tune.hip", "probe.hip", "solve.hip", "refine.hip", "kubo.hip", "adjoint.hip"]
HOST_SOURCES = ["host.cpp"]

COMMON = ["-O3", "-fPIC", "-std=c++17", "--offload-arch=gfx950", "-I" + os.path.join(HERE, "..", "include"),
          # keep the compiler from emitting packed FP32 instructions
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src, extra):
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    cmd = [HIPCC] + COMMON + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(verbose=False):
    os.makedirs(OBJ, exist_ok=True)
    jobs = [(s, []) for s in DEVICE_SOURCES if os.path.exists(os.path.join(CSRC, s))]
    # host code: no FMA contraction, so LIZ distances round exactly like plain IEEE arithmetic
    jobs += [(s, ["-ffp-contract=off"]) for s in HOST_SOURCES]
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        objs = list(ex.map(lambda a: _compile(*a), jobs))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
