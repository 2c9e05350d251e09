"""Build the HIP library librmg.so for gfx950 with hipcc (in-tree).

Every call recompiles.  Flags:
  -ffp-contract=off   no implicit FMA contraction, so the level-streaming and
                      whole-sample kernels (which share their per-cell code)
                      round identically;
  -target-feature -packed-fp32-ops
                      no packed FP32 instructions in the generated device code.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librmg.so")
SOURCES = ["solver_kernels.hip", "adjoint_kernels.hip", "kl_fields.hip", "rmg_api.cpp", "rmg_pc_mlmc.cpp"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def build(verbose: bool = False, arch: str = "gfx950", defines=(), out: str = LIB) -> str:
    """Compile every source and link ``out``; ``defines`` are extra -D tuning macros."""
    objs = []
    flags = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={arch}", "-ffp-contract=off",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument"]
    flags += [f"-D{d}" for d in defines]
    objdir = tempfile.mkdtemp(prefix="rmg_build_")
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc(), *flags, "-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd[1:1] = ["-x", "hip"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = out + ".tmp"
    cmd = [hipcc(), f"--offload-arch={arch}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    for o in objs:
        os.remove(o)
    os.rmdir(objdir)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
