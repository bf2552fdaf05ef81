"""Build of libmetade.so for gfx950 with hipcc.

Run as ``python -m paper_2502_10470_amd.build``.  The library is compiled
in-tree so it travels with the source tree.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmetade.so")
SOURCES = ["kernels.hip", "kernels_mfma.hip", "kernels_ctrl.hip", "api.hip"]
ARCH = os.environ.get("METADE_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    # DE arithmetic must be one rounding per operation (bit-exact trial vectors)
    "-ffp-contract=off",
    # no packed float32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, defines: tuple = (), tag: str = "") -> str:
    """Compile every source to its own object (in parallel), then link.  With
    a tag, the objects go to _build/<tag> and the library to
    libmetade_<tag>.so (diagnostic builds with extra -D defines)."""
    from concurrent.futures import ThreadPoolExecutor

    objdir = os.path.join(HERE, "_build", tag) if tag else os.path.join(HERE, "_build")
    out = os.path.join(HERE, f"libmetade_{tag}.so") if tag else LIB
    os.makedirs(objdir, exist_ok=True)
    compile_flags = [f for f in HIP_FLAGS if f != "-shared"] + [f"-D{d}" for d in defines]

    def compile_one(src: str) -> str:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc(), *compile_flags, "-I", os.path.join(ROOT, "include"), "-c",
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError(f"hipcc failed compiling {src}")
        return obj

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = out + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed linking {os.path.basename(out)}")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
