"""Builds libnx.so (the gfx950 HIP library behind include/nx.h) and libnx_micro.so (the
VALU issue-rate microbenchmarks behind include/nx_micro.h) in-tree with hipcc.

Every HIP source is compiled for gfx950 only, with FMA contraction off (the kernels
spell out their fused multiply-adds) and packed-FP32 instruction selection disabled.
Run ``python -m paper_1010_2641_amd.build``; ``__graft_entry__.build()`` calls it."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libnx.so")
LIB_MICRO = os.path.join(PKG, "libnx_micro.so")
BUILD = os.path.join(ROOT, "_build")
ARCH = "gfx950"

SOURCES = ["nx_fwd.hip", "nx_bwd.hip", "nx_loss.hip", "nx_species.hip", "nx_api.cpp"]
MICRO_SOURCES = ["nx_micro.hip"]

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wall", "-Wno-unused-command-line-argument",
]


def _hipcc():
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [_hipcc(), *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd.insert(1, "-xhip")
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = [l for l in (r.stderr or "").splitlines() if "packed-fp32-ops" not in l]
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n" + "\n".join(noise))
    if noise:
        print("\n".join(noise), file=sys.stderr)
    return obj


def _link(objs, lib):
    tmp = lib + ".tmp"
    r = subprocess.run([_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, lib)


def build() -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = SOURCES + MICRO_SOURCES
    with cf.ThreadPoolExecutor(max_workers=len(srcs)) as ex:
        objs = dict(zip(srcs, ex.map(_compile, srcs)))
    _link([objs[s] for s in SOURCES], LIB)
    _link([objs[s] for s in MICRO_SOURCES], LIB_MICRO)
    return LIB


if __name__ == "__main__":
    print(build())
