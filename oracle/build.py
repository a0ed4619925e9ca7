"""Build step for the oracle's shared library (test infrastructure only).

Compiles ``lbm_oracle.c`` with gcc into ``liblbm_oracle.so`` beside it, and
the same source with -fopenmp into ``liblbm_oracle_omp.so`` (its row loops on
several threads, used only to time the oracle on all host cores).  Plain -O2,
no fast-math and no FMA contraction, so the oracle's rounding follows the C
source as written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liblbm_oracle.so")
# the same source with its OpenMP row loops enabled (all-cores timing only)
LIB_OMP = os.path.join(HERE, "liblbm_oracle_omp.so")


def build(verbose=False):
    for out, extra in ((LIB, []), (LIB_OMP, ["-fopenmp"])):
        cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-Wno-unknown-pragmas",
               "-ffp-contract=off", "-fPIC", "-shared"] + extra + [SRC, "-o", out + ".tmp", "-lm"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(out + ".tmp", out)
    return LIB


def build_variant(out, defines):
    """A copy of the oracle compiled with extra -D definitions (the planted-
    mistake switches of the transport pins' own check); returns its path."""
    cmd = ["gcc", "-O2", "-std=c99", "-Wno-unknown-pragmas", "-ffp-contract=off", "-fPIC",
           "-shared"] + ["-D%s=%s" % kv for kv in sorted(defines.items())] + [SRC, "-o", out, "-lm"]
    subprocess.check_call(cmd)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
