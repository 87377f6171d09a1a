"""Build libsird.so for gfx950 with hipcc (in-tree, no JIT cache).

Flags:
  -O3 -std=c++17 --offload-arch=gfx950
  -ffp-contract=off   the swarm update must be separately rounded multiplies
                      and adds; every fused multiply-add in the kernels is an
                      explicit fma() call
  -Xclang -target-feature -Xclang -packed-fp32-ops
                      keep the compiler from emitting packed FP32 VALU ops
  -Werror=shadow      a local that shadows another is an error: kernels keep
                      many same-typed doubles in one scope, where a shadowed
                      name silently reads the wrong value

    python -m paper_2204_12346_amd.build
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsird.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Werror=shadow",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(verbose=False) -> str:
    """Compile every HIP source of the library into libsird.so."""
    out_tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + ["-I", os.path.join(ROOT, "include"), "-o", out_tmp] + sources()
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    # hipcc's host pass does not know the packed-fp32 feature and says so
    lines = [ln for ln in res.stdout.splitlines()
             if "packed-fp32-ops" not in ln and "is not a recognized feature" not in ln]
    if res.returncode != 0:
        sys.stderr.write("\n".join(lines) + "\n")
        raise RuntimeError("hipcc failed building libsird.so")
    if verbose and lines:
        print("\n".join(lines))
    os.replace(out_tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
