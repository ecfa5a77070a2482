"""Compile the gfx950 shared library libnnvisr.so in-tree with hipcc.

Usage: python -m paper_2308_03121_amd.build   (or call build()).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libnnvisr.so")
SOURCES = ["k_pixel.hip", "k_net.hip", "k_dcn.hip", "k_pyr.hip", "api.cpp"]
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Wall", "-Wno-unused-function",
    # keep the compiler from forming packed-FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{os.path.join(ROOT, 'include')}",
]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _filtered(text: str):
    # the host pass does not know the packed-fp32 feature and says so; that is harmless
    return [ln for ln in text.strip().splitlines() if "packed-fp32-ops" not in ln]


def build(verbose: bool = False) -> str:
    """Compile every source into libnnvisr.so (always rebuilds): the translation units
    are compiled in parallel into objects under _build/, then linked.  Returns the path."""
    obj_dir = os.path.join(ROOT, "_build")
    os.makedirs(obj_dir, exist_ok=True)
    compile_flags = [f for f in FLAGS if f != "-shared"]
    procs = []
    for src in SOURCES:
        obj = os.path.join(obj_dir, src + ".o")
        cmd = [hipcc()] + compile_flags + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, obj, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    objs, failed = [], []
    for cmd, obj, p in procs:
        lines = _filtered(p.communicate()[0])
        if p.returncode != 0:
            failed.append("hipcc failed: " + " ".join(cmd) + "\n" + "\n".join(lines))
        elif verbose and lines:
            print("\n".join(lines), flush=True)
        objs.append(obj)
    if failed:
        raise RuntimeError("\n".join(failed))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    lines = _filtered(res.stdout + res.stderr)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + "\n".join(lines))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
