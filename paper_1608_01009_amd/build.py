"""Build libpic_hip.so for gfx950 with hipcc (in-tree, no JIT cache).

Flags:
* ``--offload-arch=gfx950``: MI355X (CDNA4) only.
* ``-munsafe-fp-atomics``: FP64 atomic adds compile to the native
  ``global_atomic_add_f64`` / ``ds_add_f64`` instructions instead of CAS loops
  (the device memory is coarse-grained ``hipMalloc`` memory).
* ``-Xclang -target-feature -Xclang -packed-fp32-ops``: no packed FP32 math.
* no ``-ffast-math``: the push keeps IEEE division and square root.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "libpic_hip.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-munsafe-fp-atomics",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", f"-I{INCLUDE}", f"-I{CSRC}"]


# Per-source flags: the particle kernels are latency-bound at four (FP64) and six
# (FP32-mixed) waves per SIMD, where the machine scheduler's ILP strategy
# measured 0.4-0.8 % faster than the default occupancy-driven one, at the same
# register counts.
EXTRA = {
    "push_deposit.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"],
    "push_mixed.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"],
}


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(verbose: bool = False, jobs: int = 8) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    objdir = os.path.join(LIBDIR, "_obj")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = [HIPCC, *COMMON, *EXTRA.get(os.path.basename(src), []), "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _drain(procs)
    _drain(procs)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def _drain(procs):
    failed = []
    while procs:
        src, p = procs.pop(0)
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if p.returncode != 0:
            failed.append((src, text))
        elif text.strip():
            # hipcc's host pass warns about the device-only target feature
            lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l
                     and "warning generated" not in l and l.strip()]
            if lines:
                sys.stderr.write(text)
    if failed:
        for src, text in failed:
            sys.stderr.write(f"--- {src}\n{text}\n")
        raise RuntimeError("hipcc failed for " + ", ".join(os.path.basename(s) for s, _ in failed))


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
