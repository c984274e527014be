"""Build the CPU oracle library (test infrastructure, not product code).

Compiles ``pic_oracle.c`` and ``pic_oracle_adjoint.c`` with gcc into ``liborc.so`` beside this file.
``-ffp-contract=off`` keeps every expression rounding as written; no
``-ffast-math``.  Single-threaded by design.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liborc.so")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, f) for f in ("pic_oracle.c", "pic_oracle_adjoint.c")]
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", LIB + ".tmp"] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
