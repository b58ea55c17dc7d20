"""Compile tests/c_abi/step_cli (host code only) against the built libmhd.so."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
EXE = os.path.join(HERE, "step_cli")


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    pkg = os.path.join(ROOT, "paper_2511_20337_amd")
    tmp = EXE + ".tmp%d" % os.getpid()
    cmd = [hipcc, "--offload-arch=gfx950", "-O2", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), os.path.join(HERE, "step_cli.cpp"),
           "-L", pkg, "-lmhd", "-Wl,-rpath,$ORIGIN/../../paper_2511_20337_amd", "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, EXE)
    return EXE


if __name__ == "__main__":
    build(verbose=True)
