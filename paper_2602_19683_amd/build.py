"""Builds libgpr.so (all HIP sources in csrc/) for gfx950 with hipcc, in-tree.

Every source is compiled on each call (the objects go to a temporary folder),
then linked into paper_2602_19683_amd/libgpr.so. The SHA-256 of the sources
(csrc/ and include/) is compiled into the library (gpr_source_hash), so a
loader can refuse a library built from other sources.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import hashlib
import os
import shutil
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgpr.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Wall", "-Wno-unused-function",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def _sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def source_hash() -> str:
    """First 16 hex digits of the SHA-256 over every file the library is
    built from (csrc/*, include/*), by name and content, in sorted order."""
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(CSRC, "*")) + glob.glob(os.path.join(ROOT, "include", "*")))
    for f in files:
        if os.path.isfile(f):
            h.update(os.path.relpath(f, ROOT).encode())
            h.update(b"\0")
            h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def _compile(src, obj, verbose, digest):
    flags = [*FLAGS, f'-DGPR_SOURCE_HASH="{digest}"']
    cmd = [HIPCC, *flags, "-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, "-x", "hip", *flags, "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {os.path.basename(src)}:\n{err}")
    if err.strip() and verbose:
        print(err, flush=True)


def build(verbose: bool = False) -> str:
    """Compiles every source and links libgpr.so; returns its path."""
    tmp = tempfile.mkdtemp(prefix="gpr_build_")
    try:
        srcs = _sources()
        digest = source_hash()
        objs = [os.path.join(tmp, os.path.basename(s) + ".o") for s in srcs]
        with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
            list(ex.map(lambda so: _compile(so[0], so[1], verbose, digest), zip(srcs, objs)))
        out_tmp = LIB + ".tmp"
        # roctx: the marker ranges of each entry point and launch group
        cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", out_tmp,
               "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(out_tmp, LIB)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
