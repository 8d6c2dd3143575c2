"""Build libbingo.so for gfx950 with hipcc (in-tree, next to this file).

Each source compiles to its own object in parallel (no device code crosses a translation unit),
then one hipcc call links the shared library."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["api.hip", "prim.hip", "build.hip", "walk.hip", "export.hip", "update.hip", "serve.hip", "probe.hip", "stream.hip",
           "node2vec.hip", "compact.hip", "radix4.hip", "locate.hip"]
OUT = os.path.join(HERE, "libbingo.so")
OBJ_DIR = os.path.join(HERE, "_build")
FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-value", "-Wno-unused-result",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
    return r.returncode


def build(verbose: bool = False, jobs: int = 0) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ_DIR, exist_ok=True)
    inc = "-I" + os.path.join(ROOT, "include")
    objs, cmds = [], []
    for s in SOURCES:
        o = os.path.join(OBJ_DIR, s.replace(".hip", ".o"))
        objs.append(o)
        cmds.append([hipcc] + FLAGS + [inc, "-c", "-o", o, os.path.join(HERE, "csrc", s)])
    jobs = jobs or min(len(cmds), max(1, min(os.cpu_count() or 1, 16)))
    with ThreadPoolExecutor(jobs) as ex:
        rcs = list(ex.map(lambda c: _run(c, verbose), cmds))
    if any(rcs):
        raise RuntimeError("hipcc failed compiling libbingo sources")
    tmp = OUT + ".tmp%d" % os.getpid()
    if _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs, verbose):
        raise RuntimeError("hipcc failed linking libbingo.so")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
