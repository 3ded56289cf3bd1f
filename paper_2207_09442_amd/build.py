"""Build step of the HIP library: compiles csrc/*.hip for gfx950 into
libdnls.so next to this file (in-tree, so that it ships with the source)."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libdnls.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("dnls.hip", "ba.hip", "sparse.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # packed FP32 instructions are disabled: some of their forms have been
    # observed to return wrong results on this hardware
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libdnls.so")


def build(verbose: bool = False) -> str:
    """Compile the library (always: each source to an object, in parallel,
    then one shared-library link) and return its path."""
    objs = [os.path.join(HERE, os.path.basename(src) + ".o") for src in SOURCES]
    cmds = [[HIPCC, *FLAGS, "-c", "-o", o, src] for src, o in zip(SOURCES, objs)]
    with ThreadPoolExecutor(len(cmds)) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
    for o in objs:
        os.remove(o)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
