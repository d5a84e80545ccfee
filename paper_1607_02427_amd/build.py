"""Builds libdem.so (HIP, gfx950) in-tree from csrc/*.hip.

Every HIP source is compiled with packed-FP32 instructions disabled (the
compiler would otherwise form v_pk_* FP32 operations on its own)."""
import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libdem.so")
SOURCES = ["dem_lists.hip", "dem_force.hip", "dem_integrate.hip", "dem_runtime.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def resources_path(src: str) -> str:
    """The compiler's per-kernel resource report (registers, scratch, LDS,
    occupancy) for one source, written by the last build."""
    return os.path.join(BUILD, src.replace(".hip", ".resources.txt"))


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, src.replace(".hip", ".o"))
    cmd = [HIPCC] + FLAGS + ["-Rpass-analysis=kernel-resource-usage", "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stderr=subprocess.PIPE, text=True)
    with open(resources_path(src), "w") as f:
        f.write(r.stderr)
    # pass warnings and errors through; the resource remarks go to the file
    rest = [ln for ln in r.stderr.splitlines() if "remark:" not in ln and not re.match(r"\s*\d*\s*\|", ln)]
    if rest:
        print("\n".join(rest), file=sys.stderr, flush=True)
    if r.returncode != 0:
        raise subprocess.CalledProcessError(r.returncode, cmd)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(4, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
