"""Build libsv.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2402_15281_amd.build [--asm]

Every translation unit under csrc/ is compiled for gfx950 only and linked into
paper_2402_15281_amd/libsv.so.  Packed FP32 instructions are disabled for all
device code; hipcc's host pass reports that it does not know that feature,
which is harmless.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsv.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["sv_api.hip", "sv_geom.hip", "sv_batch.hip", "sv_search.hip", "sv_cull.hip", "sv_mlp.hip", "sv_train.hip"]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
    "-Wno-unused-result",
]


def _compile(src: str, asm: bool):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    if asm:
        cmd += ["-save-temps=obj"]
    return obj, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)


def build(asm: bool = False, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = [_compile(s, asm) for s in SOURCES]
    objs, failed = [], []
    for obj, p in jobs:
        out, _ = p.communicate()
        noise = [ln for ln in out.splitlines() if "packed-fp32-ops" not in ln and "warnings generated" not in ln]
        if p.returncode != 0:
            failed.append((obj, out))
        elif verbose and noise:
            print("\n".join(noise))
        objs.append(obj)
    if failed:
        for obj, out in failed:
            sys.stderr.write(f"--- {obj}\n{out}\n")
        raise RuntimeError("hipcc failed")
    tmp = LIB + ".tmp"
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp], check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(asm="--asm" in sys.argv, verbose=True))
