"""Build the native parts in-tree.

* ``libyoro.so``: the HIP kernels and the C-ABI (``include/yoro.h``), built
  with hipcc for gfx950 only.
* ``scenes/libyoro_scene.so``: the seeded scene generator and ray-caster
  (gcc, OpenMP).

Flags: ``-ffp-contract=off`` on every compile so that each FP32 operation
rounds once, as written; packed FP32 instructions are disabled for the device
code; no fast-math anywhere.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB_YORO = os.path.join(HERE, "libyoro.so")
LIB_SCENE = os.path.join(HERE, "scenes", "libyoro_scene.so")
BUILD_DIR = os.path.join(ROOT, "_build")

ARCH = "gfx950"
HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    f"-I{INCLUDE}",
]


def _hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd):
    print("+", " ".join(cmd), file=sys.stderr, flush=True)
    subprocess.check_call(cmd)


def hip_sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def build_yoro(jobs: int = 8) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    objs = []
    procs = []
    for src in hip_sources():
        obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = [_hipcc(), *HIPCC_FLAGS, "-c", src, "-o", obj]
        print("+", " ".join(cmd), file=sys.stderr, flush=True)
        procs.append(subprocess.Popen(cmd, stderr=subprocess.PIPE, text=True))
        if len(procs) >= jobs:
            _wait(procs)
            procs = []
    _wait(procs)
    tmp = LIB_YORO + ".tmp"
    _run([_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIB_YORO)
    return LIB_YORO


def _wait(procs):
    failed = False
    for p in procs:
        _, err = p.communicate()
        # hipcc's host pass does not know the device-only feature flag; drop that noise.
        lines = [ln for ln in (err or "").splitlines() if "packed-fp32-ops" not in ln]
        if lines:
            print("\n".join(lines), file=sys.stderr)
        if p.returncode != 0:
            failed = True
    if failed:
        raise RuntimeError("hipcc failed")


def build_scene() -> str:
    src = os.path.join(HERE, "scenes", "raycast.c")
    tmp = LIB_SCENE + ".tmp"
    _run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-Wall",
          src, "-o", tmp, "-lm"])
    os.replace(tmp, LIB_SCENE)
    return LIB_SCENE


def build_all() -> None:
    build_scene()
    build_yoro()


if __name__ == "__main__":
    build_all()
