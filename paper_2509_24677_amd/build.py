"""Build of the gfx950 HIP library ``libneuralpvs.so`` (in-tree, next to this file).

Every ``csrc/*.hip`` source is compiled for gfx950 only, in parallel, and linked into one shared
library that exports the C ABI of ``include/neuralpvs.h``.
"""
from __future__ import annotations

import glob
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libneuralpvs.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def sources():
    return sorted(glob.glob(os.path.join(SRC, "*.hip")))


def source_hash() -> str:
    """16 hex digits of SHA-256 over every file the library is built from (csrc/*.hip, csrc/*.hpp,
    include/neuralpvs.h) and the compile flags; compiled into the library (npvs_source_hash) so
    the loader can refuse a library built from other sources."""
    h = hashlib.sha256(" ".join(FLAGS).encode())
    files = sources() + sorted(glob.glob(os.path.join(SRC, "*.hpp")))
    files.append(os.path.join(os.path.dirname(HERE), "include", "neuralpvs.h"))
    for f in files:
        h.update(os.path.basename(f).encode() + b"\0")
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def build(verbose: bool = False) -> str:
    os.makedirs(OUT, exist_ok=True)
    procs = []
    objs = []
    tag = f'-DNPVS_SOURCE_HASH="{source_hash()}"'
    for src in sources():
        obj = os.path.join(OUT, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = [HIPCC, *FLAGS, tag, "-c", src, "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    errors = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # the host pass does not know the packed-fp32 feature; that warning is harmless
        lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln]
        if p.returncode != 0:
            errors.append(f"{src}:\n" + "\n".join(lines))
        elif verbose and lines:
            print("\n".join(lines), file=sys.stderr)
    if errors:
        raise RuntimeError("HIP build failed:\n" + "\n".join(errors))
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
