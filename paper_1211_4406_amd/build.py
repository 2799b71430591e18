"""Build libsrf.so (HIP, gfx950) in place.

    python paper_1211_4406_amd/build.py

(run as a script: importing the package loads the library it builds).  It also
builds libsrf_calib.so, the vector-ALU issue-rate calibration that
`bench.py --valu-calibration` runs.

Every translation unit is compiled for gfx950 only, with packed FP32
instructions disabled.  The cell/group and list units are compiled without
floating-point contraction because the tree decisions must be the literal
FP64 expressions.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsrf.so")
# the vector-ALU issue-rate calibration (a measurement tool, its own library)
CALIB_SRC = os.path.join(HERE, "calib", "valu_issue.hip")
CALIB_LIB = os.path.join(HERE, "libsrf_calib.so")

SOURCES = {
    "runtime.hip": [],
    "sort.hip": [],
    "tree.hip": ["-ffp-contract=off"],
    "lists.hip": ["-ffp-contract=off"],
    "pair.hip": [],
    "quad.hip": [],
    "pm.hip": [],
    "integ.hip": [],
    "api.hip": [],
}

COMMON = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str, extra: list[str], save_temps: bool) -> str:
    obj = os.path.join(BUILD, src.replace(".hip", ".o"))
    cmd = [hipcc(), *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    if save_temps:
        cmd += ["--save-temps"]
    r = subprocess.run(cmd, cwd=BUILD, capture_output=True, text=True)
    msg = "\n".join(line for line in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in line)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{msg}")
    if msg.strip():
        print(msg, file=sys.stderr)
    return obj


def build(save_temps: bool = False, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(lambda kv: _compile(kv[0], kv[1], save_temps), SOURCES.items()))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    tmp = CALIB_LIB + ".tmp"
    r = subprocess.run([hipcc(), *COMMON, "-shared", "-o", tmp, CALIB_SRC], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("calibration library failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, CALIB_LIB)
    if verbose:
        print("built", LIB, "and", CALIB_LIB)
    return LIB


if __name__ == "__main__":
    build(save_temps="--save-temps" in sys.argv, verbose=True)
