"""Compile libnexels.so for gfx950 with hipcc (in-tree, no JIT cache).

    python paper_2512_13796_amd/build.py   (run as a script: importing the package
                                           would load the library it builds)
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libnexels.so")
SOURCES = ["api.hip", "preprocess.hip", "sort.hip", "raster.hip", "texture.hip", "aux.hip", "adc.hip"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags() -> list:
    return [
        "--offload-arch=gfx950",
        "-O3",
        "-std=c++17",
        "-fPIC",
        "-ffp-contract=on",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I" + os.path.join(ROOT, "include"),
        "-Wno-unused-result",
    ]


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every source to an object in parallel, then link the shared library."""
    cc = hipcc()
    tmp = tempfile.mkdtemp(prefix="nx_build_")
    procs = []
    objs = []
    try:
        for src in SOURCES:
            obj = os.path.join(tmp, src.replace(".hip", ".o"))
            objs.append(obj)
            cmd = [cc, *flags(), "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
            while sum(p.poll() is None for _, p in procs) >= jobs:
                procs[[p.poll() is None for _, p in procs].index(True)][1].wait()
        failed = []
        for src, p in procs:
            out, _ = p.communicate()
            text = out.decode(errors="replace")
            lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln]
            if p.returncode != 0:
                failed.append((src, "\n".join(lines)))
            elif verbose and lines:
                print("\n".join(lines))
        if failed:
            msg = "\n\n".join(f"--- {s}\n{t}" for s, t in failed)
            raise RuntimeError("hipcc failed:\n" + msg)
        tmp_lib = LIB + ".tmp"
        cmd = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp_lib]
        subprocess.run(cmd, check=True, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
        os.replace(tmp_lib, LIB)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    path = build(verbose="-v" in sys.argv)
    print(path)
