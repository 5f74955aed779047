"""Builds libesom.so (HIP, gfx950) in-tree with hipcc.

Every build compiles from source; objects go to ``_build/`` next to this file
and the shared library to ``libesom.so``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libesom.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
ARCH = os.environ.get("ESOM_OFFLOAD_ARCH", "gfx950")

FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
         # keep hipcc from forming packed FP32 instructions (v_pk_*_f32)
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", INCLUDE, "-I", CSRC]

UNITS = [("esom_core.hip", []), ("esom_update.hip", []), ("esom_api.cpp", ["-x", "hip"]),
         ("esom_serve.cpp", ["-x", "hip"]), ("esom_som.hip", []), ("esom_graph.hip", []),
         ("esom_embed3.hip", []), ("esom_ablation.hip", []),
         ("esom_materialise.hip", []), ("esom_bin.hip", [])]
for mode in (0, 1):
    for kp in (8, 16, 20, 24, 32):
        UNITS.append(("embed_inst.hip", ["-DINST_MODE=%d" % mode, "-DINST_KP=%d" % kp, "-DINST_KF=0"]))
        if kp != 24:
            UNITS.append(("embed_inst.hip", ["-DINST_MODE=%d" % mode, "-DINST_KP=%d" % kp, "-DINST_KF=1"]))


def _obj_name(src, defs):
    stem = os.path.splitext(src)[0]
    tag = "".join(d.split("=")[1] for d in defs if d.startswith("-D"))
    return os.path.join(BUILD, stem + ("_" + tag if tag else "") + ".o")


def _compile(unit):
    src, extra = unit
    obj = _obj_name(src, extra)
    cmd = ["hipcc"] + FLAGS + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                     if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, msgs))
    return obj


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(8, max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, UNITS))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc", "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
