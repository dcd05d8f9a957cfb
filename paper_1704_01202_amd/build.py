"""Builds the HIP library libxpic.so for gfx950 in-tree (hipcc, no JIT cache).

FP64 arithmetic follows the library's arithmetic contract: no contraction of
products into fused multiply-adds (-ffp-contract=off) and no fast-math; packed
FP32 instructions are disabled.
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libxpic.so")
SOURCES = ["xp_api.hip", "xp_step.hip", "xp_big.hip", "xp_bin.hip", "xp_diag.hip", "xp_rad.hip"]
ARCH = os.environ.get("XPIC_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "--offload-arch=" + ARCH, "-fPIC", "-ffp-contract=off",
         "-fno-fast-math", "-Werror=return-type", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result"]


def build(verbose=False, jobs=4):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [hipcc, "-c", *FLAGS, "-o", obj, os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _wait(procs)
            procs = []
    _wait(procs)
    tmp = LIB + ".tmp"
    cmd = [hipcc, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp, *objs]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout.decode())
    os.replace(tmp, LIB)
    return LIB


def _wait(procs):
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode()
        if p.returncode != 0:
            raise RuntimeError("hipcc failed on %s:\n%s" % (src, text))


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
