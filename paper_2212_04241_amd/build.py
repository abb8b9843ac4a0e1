"""Build the HIP library libfbn.so in-tree for gfx950 with hipcc.

Usage: python -m paper_2212_04241_amd.build
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libfbn.so")

SOURCES = ["kernels.hip", "kernels_interleaved.hip", "kernels_query.hip", "api.cpp", "tree.cpp", "plan.cpp", "bif.cpp"]
ARCH = os.environ.get("FBN_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags(src: str) -> list:
    f = ["-O3", "-std=c++17", "-fPIC", "-Wall", f"--offload-arch={ARCH}",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC,
         # packed fp32 instructions stay off: some of their forms have given
         # wrong results on this hardware without any error
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    if src.endswith(".hip"):
        f += ["-x", "hip"]
    return f


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    cc = hipcc()
    procs = []
    objs = []
    for s in SOURCES:
        obj = os.path.join(BUILD, s.replace(".", "_") + ".o")
        cmd = [cc] + flags(s) + ["-c", os.path.join(CSRC, s), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((s, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        objs.append(obj)
    failed = []
    for s, p in procs:
        out, _ = p.communicate()
        lines = [ln for ln in out.splitlines() if "packed-fp32-ops" not in ln]
        if p.returncode != 0:
            failed.append((s, "\n".join(lines)))
        elif verbose and lines:
            print("\n".join(lines))
    if failed:
        raise RuntimeError("\n".join(f"--- {s}\n{msg}" for s, msg in failed))
    tmp = LIB + ".tmp"
    cmd = [cc, "-shared", f"--offload-arch={ARCH}", "-o", tmp] + objs
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
