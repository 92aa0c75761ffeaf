"""Builds libsrtm.so (the HIP kernels and the C-ABI host code) in-tree for gfx950."""
from __future__ import annotations

import os
import re
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsrtm.so")
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")


def pairs():
    """The (nx, ny) pairs listed in SRTM_PAIRS (csrc/srtm_entry.h)."""
    text = open(os.path.join(CSRC, "srtm_entry.h")).read()
    line = re.search(r"#define SRTM_PAIRS\(X\)(.*)", text).group(1)
    return [(int(a), int(b)) for a, b in re.findall(r"X\((\d+),\s*(\d+)\)", line)]


def units():
    """(source, extra flags, object name): the host ABI code, the kernels once per pair, and the
    mixed-pair batch kernels once per element type."""
    out = [("srtm_api.hip", [], "srtm_api.o")]
    for a, b in pairs():
        out.append(("srtm_kernels.hip", [f"-DSRTM_NX={a}", f"-DSRTM_NY={b}"], f"srtm_kernels_{a}_{b}.o"))
    for t in ("double", "float"):  # the mixed-pair batch kernels, once per element type
        out.append(("srtm_kernels.hip", [f"-DSRTM_MIXED_T={t}"], f"srtm_kernels_mixed_{t}.o"))
    return out

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay off (hipcc would otherwise form them from float code)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False) -> str:
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)

    def compile_one(unit):
        src, extra, obj_name = unit
        obj = os.path.join(build_dir, obj_name)
        cmd = [HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        return obj, r, src

    jobs = max(1, min(len(units()), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(compile_one, units()))
    objs = []
    for obj, r, src in results:
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError(f"hipcc failed on {src} ({os.path.basename(obj)})")
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link of libsrtm.so failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
