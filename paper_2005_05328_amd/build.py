"""Build libdzs.so (gfx950) in-tree with hipcc.

Every translation unit is compiled with -ffp-contract=off so that the exact paths (keys,
drift, lightcone selection, DZS node sums and predicate) round every operation as written,
and with packed-FP32 instructions disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libdzs.so")
BUILD_DIR = os.path.join(HERE, "_build")
SOURCES = ["abi.hip", "sort.hip", "particles.hip", "tree.hip", "pm.hip", "coarsen.hip",
           "cosmo.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument", "-I", os.path.join(HERE, "..", "include")]


def source_hash() -> str:
    """SHA-256 (first 16 hex digits) of everything the library is built from: the HIP and C++
    sources and internal headers, the public header and this build script (its flags).  The
    binding recomputes it at import and refuses a library built from other sources."""
    h = hashlib.sha256()
    files = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp", ".h")))
    paths = [os.path.join(CSRC, f) for f in files]
    paths += [os.path.join(HERE, "..", "include", "dzs.h"), os.path.abspath(__file__)]
    for path in paths:
        h.update(os.path.basename(path).encode())
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _compile(src: str, digest: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, f'-DDZS_SOURCE_HASH="{digest}"', "-c", os.path.join(CSRC, src), "-o",
           obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, "-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-I",
               os.path.join(HERE, "..", "include"), f'-DDZS_SOURCE_HASH="{digest}"', "-c",
               os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 4)) as ex:
        digest = source_hash()
        objs = list(ex.map(lambda src: _compile(src, digest), SOURCES))
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
