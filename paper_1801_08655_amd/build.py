"""Build the HIP library ``libhelm.so`` in-tree for gfx950.

Every source under ``csrc/`` is compiled with hipcc (HIP for gfx950; the
packed-FP32 instructions are disabled) and linked into one shared library
next to this file.  ``build()`` always recompiles what changed.
"""

from __future__ import annotations

import concurrent.futures
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhelm.so")
ARCH = os.environ.get("HELM_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-Wno-unused-command-line-argument",
]


def _sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def _headers_digest():
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        if f.endswith(".h"):
            with open(os.path.join(CSRC, f), "rb") as fh:
                h.update(fh.read())
    inc = os.path.join(HERE, "..", "include")
    for f in sorted(os.listdir(inc)):
        if f.endswith(".h"):
            with open(os.path.join(inc, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def _compile(src, hdr):
    path = os.path.join(CSRC, src)
    with open(path, "rb") as fh:
        digest = hashlib.sha256(fh.read() + hdr.encode() + " ".join(FLAGS).encode()).hexdigest()[:16]
    obj = os.path.join(BUILD, f"{src}.{digest}.o")
    if os.path.exists(obj):
        return obj
    cmd = ["hipcc", *FLAGS, "-x", "hip", "-c", path, "-o", obj + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    os.replace(obj + ".tmp", obj)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hdr = _headers_digest()
    srcs = _sources()
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, hdr), srcs))
    cmd = ["hipcc", *FLAGS, "-shared", *objs, "-o", LIB + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-6000:]}")
    os.replace(LIB + ".tmp", LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
