"""Build libmtvd.so (HIP, gfx950) in-tree with hipcc.

Every HIP source under csrc/ is compiled for gfx950 with packed-FP32
instructions disabled and linked into one shared library next to this file.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmtvd.so")
ARCH = os.environ.get("MTVD_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


# Instruction-scheduling strategy per source, chosen by timing the step at
# 4096x1024 and 1024x1024x256 (it only reorders instructions: results are
# bit for bit the same).  The 2D sweeps gained 2% with max-ilp; the 3D
# march kernels 1.4% with iterative-minreg; the rest keep the default.
SCHED = {
    "mtvd_2d.hip": "max-ilp",
    "mtvd_3d_x.hip": "iterative-minreg",
    "mtvd_3d_y.hip": "iterative-minreg",
    "mtvd_3d_z.hip": "iterative-minreg",
}

# The 3D L_z operator runs its plate rows and the rows between in two
# separately compiled copies of the same arithmetic; with multiply-adds
# fused where the compiler likes, the copies rounded differently, so a
# node's last bits depended on which copy its chunk ran (on the rows per
# wave).  Without fusion every expression rounds as written in both copies.
# (L_x and L_y have one copy each and keep their fused multiply-adds.)
EXTRA = {
    "mtvd_3d_z.hip": ["-ffp-contract=off"],
}


def flags_for(src: str) -> list:
    name = os.path.basename(src)
    st = SCHED.get(name)
    return (FLAGS + (["-mllvm", f"-amdgpu-sched-strategy={st}"] if st else [])
            + EXTRA.get(name, []))


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    for src in sources():
        obj = os.path.join(HERE, "_build", os.path.basename(src) + ".o")
        cmd = [hipcc, *flags_for(src), "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
