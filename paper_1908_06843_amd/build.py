"""Build libprosper.so (HIP, gfx950) in-tree.

    python -m paper_1908_06843_amd.build [-v] [--incremental]

Every .hip file under csrc/ is compiled to an object under _build/ (in
parallel) and linked into paper_1908_06843_amd/libprosper.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libprosper.so")

ARCH = os.environ.get("PROSPER_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # keep the backend from forming packed FP32 ops on its own
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _local_includes(path: str, seen: set) -> None:
    """Every project header `path` includes, transitively (quoted includes)."""
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if line.startswith("#include") and '"' in line:
                name = line.split('"')[1]
                for d in (CSRC, INCLUDE):
                    f = os.path.join(d, name)
                    if os.path.exists(f) and f not in seen:
                        seen.add(f)
                        _local_includes(f, seen)


def _key(src: str) -> str:
    """Hash of a source, the project headers it includes and the flags."""
    h = hashlib.sha256(" ".join([HIPCC, *FLAGS]).encode())
    seen: set = set()
    _local_includes(src, seen)
    for f in [src, *sorted(seen)]:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _compile(src: str, verbose: bool, incremental: bool) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    key = _key(src)
    stamp = obj + ".key"
    if incremental and os.path.exists(obj) and os.path.exists(stamp):
        with open(stamp) as fh:
            if fh.read() == key:
                return obj
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{r.stdout}\n{r.stderr}")
    with open(stamp, "w") as fh:
        fh.write(key)
    return obj


def build(verbose: bool = False, jobs: int = 8, incremental: bool = False) -> str:
    """Compile every source (incremental=True reuses objects whose source,
    headers and flags are unchanged) and link the library."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(jobs, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, incremental), srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv))
