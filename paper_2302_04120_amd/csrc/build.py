"""Build step of liblbm.so: hipcc for gfx950, in-tree.

Compiles the HIP sources of this directory into ``../liblbm.so``.  Only the
``extern "C"`` entry points of include/lbm.h are exported.  Packed-FP32
instructions are disabled for all device code.  Multiply-adds are fused only
within one source expression (-ffp-contract=on), never across statements:
the fusion then depends on the source alone, so kernels that inline the same
per-node function round identically.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "liblbm.so")
SOURCES = ["lbm_api.hip", "lbm_kernels.hip", "lbm_adjoint.hip", "lbm_d3q19.hip", "lbm_phase3d.hip"]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


def build(verbose=False, extra=()):
    cmd = [hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-fvisibility=hidden", "-ffp-contract=on",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I" + os.path.join(ROOT, "include"), "-I" + HERE]
    cmd += list(extra)
    cmd += [os.path.join(HERE, s) for s in SOURCES]
    cmd += ["-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


PROBE_SRC = os.path.join(HERE, "hbm_probe.hip")
PROBE_LIB = os.path.join(PKG, "libhbm_probe.so")


def build_probe(verbose=False):
    """The HBM bandwidth probe of bench.py --copy-ceiling (a library of its
    own: measurement code, not part of liblbm)."""
    cmd = [hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-fvisibility=hidden", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           PROBE_SRC, "-o", PROBE_LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(PROBE_LIB + ".tmp", PROBE_LIB)
    return PROBE_LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
