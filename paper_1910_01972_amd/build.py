"""Build the gfx950 HIP library (libols.so) and the host emulator (libols_emu.so) in-tree.

Run ``python -m paper_1910_01972_amd.build`` (or ``__graft_entry__.build()``).
Every call recompiles.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIBDIR = os.path.join(PKG, "lib")
ARCH = "gfx950"

# Packed FP32 instructions are disabled for all device code on purpose.
COMMON = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{os.path.join(ROOT, 'include')}",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout)
        raise RuntimeError(f"build failed: {' '.join(cmd)}")
    return r.stdout


def build(verbose: bool = False) -> dict:
    os.makedirs(LIBDIR, exist_ok=True)
    out = {}
    lib = os.path.join(LIBDIR, "libols.so")
    tmp = lib + ".tmp"
    _run([hipcc(), f"--offload-arch={ARCH}", *COMMON, "-o", tmp, os.path.join(CSRC, "ols_kernels.hip")], verbose)
    os.replace(tmp, lib)
    out["libols"] = lib
    emu = os.path.join(LIBDIR, "libols_emu.so")
    tmp = emu + ".tmp"
    _run([hipcc(), "-x", "hip", "--offload-host-only", *COMMON, "-o", tmp, os.path.join(CSRC, "ols_emu.cpp")], verbose)
    os.replace(tmp, emu)
    out["libols_emu"] = emu
    return out


if __name__ == "__main__":
    print(build(verbose=True))
