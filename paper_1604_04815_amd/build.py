"""Build the HIP scan library ``liblscan.so`` in-tree for gfx950.

Every ``csrc/*.hip`` unit and the host runtime are compiled with hipcc in
parallel into ``_build/`` and linked into ``paper_1604_04815_amd/liblscan.so``.
Run as ``python -m paper_1604_04815_amd.build``.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "liblscan.so")
# A user-operator scan built, as a user would, from include/lscan_custom.hpp
# into a library of its own (run through lscan_scan_custom).
CUSTOM_SRC = os.path.join(PKG, "custom", "affine_scan.hip")
CUSTOM_LIB = os.path.join(PKG, "custom", "libaffine_scan.so")
# Streaming copies of the scan's structure (persistent cyclic) and of a flat
# grid: the practical ceiling the benchmark measures beside the scan.
CEILING_SRC = os.path.join(PKG, "ceiling", "copy_ceiling.hip")
CEILING_LIB = os.path.join(PKG, "ceiling", "libcopy_ceiling.so")
INCLUDE = os.path.join(ROOT, "include")

ARCH = "gfx950"
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

# Packed-FP32 instructions are kept out of every device build: the compiler
# would otherwise form them from ordinary float code.
COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *COMMON, "-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, *COMMON, "-x", "hip", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in (r.stderr or "").splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{err}")
    return obj


def sources() -> list[str]:
    return sorted(glob.glob(os.path.join(CSRC, "*.hip"))) + sorted(glob.glob(os.path.join(CSRC, "*.cpp")))


def _link(objs: list[str], out: str) -> None:
    tmp = out + ".tmp"
    r = subprocess.run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed for {out}:\n{r.stderr}")
    os.replace(tmp, out)


def build(jobs: int | None = None, verbose: bool = False) -> str:
    """Compile every unit and link the shared library (and the user-operator
    example and copy-ceiling libraries); returns the main library's path."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(16, os.cpu_count() or 4, len(srcs) + 1)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, srcs + [CUSTOM_SRC, CEILING_SRC]))
    _link(objs[:-2], LIB)
    _link(objs[-2:-1], CUSTOM_LIB)
    _link(objs[-1:], CEILING_LIB)
    if verbose:
        print(f"built {LIB} from {len(srcs)} units, {CUSTOM_LIB} and {CEILING_LIB}", flush=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
