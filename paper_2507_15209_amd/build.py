"""Build the gfx950 shared library ``libmp3.so`` in-tree with hipcc.

Device code (kernels.hip) is compiled for gfx950 only; the C ABI and the
float64 table generation are host C++.  Objects go to ``_build/`` at the
repository root, the library next to this file.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libmp3.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", "-I", os.path.join(ROOT, "include"), "-I", CSRC]
HOST = ["-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include"]
# device code: gfx950, and no packed-FP32 instructions
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def commands() -> list[list[str]]:
    objs = []
    cmds = []
    for src, dev in (("kernels.hip", True), ("stats.hip", True), ("stencil.hip", True), ("static_scratch.hip", True),
                     ("mp3_api.cpp", False),
                     ("tables.cpp", False)):
        obj = os.path.join(BUILD, src + ".o")
        flags = COMMON + (DEVICE + ["-x", "hip"] if dev else HOST + ["-x", "c++"])
        cmds.append([HIPCC] + flags + ["-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    cmds.append([HIPCC, "-shared", f"--offload-arch={ARCH}", "-fPIC"] + objs + ["-lpthread", "-o", LIB + ".tmp"])
    return cmds


def build(verbose: bool = False) -> str:
    """Compile every source (in parallel), then link."""
    os.makedirs(BUILD, exist_ok=True)
    cmds = commands()
    procs = []
    for cmd in cmds[:-1]:
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    failed = None
    for cmd, pr in procs:
        out, _ = pr.communicate()
        if pr.returncode != 0:
            sys.stderr.write(out)
            failed = failed or cmd
    if failed:
        raise RuntimeError("hipcc failed: " + " ".join(failed[-3:]))
    if verbose:
        print(" ".join(cmds[-1]), flush=True)
    r = subprocess.run(cmds[-1], capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
