"""Builds liboceansim.so (gfx950) in-tree with hipcc.

    python paper_2503_01074_amd/build.py [--force]

Run it as a script (or load it by path): importing the package first would
load the library this script rebuilds.
"""
from __future__ import annotations

import concurrent.futures as cf
import json
import os
import re
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "liboceansim.so")
SOURCES = ["api.cpp", "plan.cpp", "bvh.cpp", "sonar.hip", "uw.hip", "cam.hip", "nav.hip", "raycast.hip"]
HEADERS = ["device.hpp", "launch.hpp", "host.hpp", "uw_body.hpp", "reduce_body.hpp", "scene.hpp"]
ARCH = os.environ.get("OCEANSIM_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-x", "hip", "-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions are left to nothing: keep the compiler from forming them
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    "-I", os.path.join(ROOT, "include"),
]


def _stale(obj: str, src: str) -> bool:
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [src] + [os.path.join(CSRC, h) for h in HEADERS] + [os.path.join(ROOT, "include", "oceansim.h")]
    return any(os.path.getmtime(d) > t for d in deps)


RESOURCE_KEYS = {"VGPRs": "vgprs", "ScratchSize [bytes/lane]": "scratch_bytes_per_lane",
                 "Occupancy [waves/SIMD]": "waves_per_simd", "LDS Size [bytes/block]": "lds_bytes",
                 "VGPRs Spill": "vgpr_spills"}


def kernel_resources(remarks: str) -> dict:
    """Per-kernel register, stack, occupancy and LDS figures from the
    compiler's kernel-resource-usage remarks (device code built here)."""
    out, cur = {}, None
    for line in remarks.splitlines():
        m = re.search(r"remark:\s+(.+?):\s+(\S+)\s+\[-Rpass-analysis", line)
        if not m:
            continue
        key, val = m.group(1).strip(), m.group(2)
        if key == "Function Name":
            cur = out.setdefault(val, {})
        elif cur is not None and key in RESOURCE_KEYS:
            cur[RESOURCE_KEYS[key]] = int(val)
    return out


def _compile(src: str, force: bool) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + ".o")
    if force or _stale(obj, path):
        cmd = [HIPCC] + FLAGS + ["-c", path, "-o", obj]
        if src.endswith(".hip"):
            cmd.append("-Rpass-analysis=kernel-resource-usage")
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, r.stdout, r.stderr))
        if src.endswith(".hip"):
            with open(os.path.join(BUILD, src + ".resources.json"), "w") as fh:
                json.dump(kernel_resources(r.stderr), fh, indent=1, sort_keys=True)
    return obj


def build(force: bool = True) -> str:
    """Compile every HIP source for gfx950 and link the shared library."""
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, force), SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--force" in sys.argv))
