"""Build steps for the native parts of the package.

* ``libgraphgen.so`` -- the seeded input generators (plain C, gcc, OpenMP).
* ``libcoop.so``     -- the cooperative-kernel runtime: hand-written HIP
  kernels for gfx950 plus the host runtime behind the C ABI in
  ``include/coop.h``.

Everything is built in-tree under ``paper_1707_01989_amd/lib`` so the
shared objects travel with the source tree.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG_DIR = os.path.dirname(os.path.abspath(__file__))
REPO_DIR = os.path.dirname(PKG_DIR)
CSRC = os.path.join(PKG_DIR, "csrc")
LIB_DIR = os.path.join(PKG_DIR, "lib")
INCLUDE_DIR = os.path.join(REPO_DIR, "include")

GRAPHGEN_SO = os.path.join(LIB_DIR, "libgraphgen.so")
COOP_SO = os.path.join(LIB_DIR, "libcoop.so")

HIP_SOURCES = ["coop_kernels.hip", "batch_kernels.hip", "serve_kernels.hip", "octree_kernels.hip",
               "cc_kernels.hip", "graph_prep.hip", "coop_runtime.hip"]
HIP_ARCH = "gfx950"


def _run(cmd: list[str]) -> None:
    print("+", " ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build_graphgen() -> str:
    os.makedirs(LIB_DIR, exist_ok=True)
    tmp = GRAPHGEN_SO + ".tmp"
    _run(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11",
          os.path.join(CSRC, "graphgen.c"), "-o", tmp, "-lm"])
    os.replace(tmp, GRAPHGEN_SO)
    return GRAPHGEN_SO


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def build_coop(jobs: int = 4) -> str:
    """Compile every HIP source for gfx950 and link libcoop.so."""
    os.makedirs(LIB_DIR, exist_ok=True)
    objdir = os.path.join(LIB_DIR, "obj")
    os.makedirs(objdir, exist_ok=True)
    cc = hipcc()
    common = [
        f"--offload-arch={HIP_ARCH}", "-O3", "-fPIC", "-std=c++17",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", INCLUDE_DIR, "-I", CSRC, "-Wall", "-Wno-unused-function",
    ]
    procs = []
    objs = []
    for src in HIP_SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        cmd = [cc, *common, "-c", os.path.join(CSRC, src), "-o", obj]
        print("+", " ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        if len(procs) >= jobs:
            for p in procs:
                if p.wait() != 0:
                    raise subprocess.CalledProcessError(p.returncode, p.args)
            procs = []
    for p in procs:
        if p.wait() != 0:
            raise subprocess.CalledProcessError(p.returncode, p.args)
    tmp = COOP_SO + ".tmp"
    _run([cc, f"--offload-arch={HIP_ARCH}", "-shared", "-fPIC", *objs, "-o", tmp,
          "-lpthread", "-Wl,--no-undefined"])
    os.replace(tmp, COOP_SO)
    return COOP_SO


def build_all() -> None:
    build_graphgen()
    build_coop()


if __name__ == "__main__":
    what = sys.argv[1:] or ["all"]
    for w in what:
        {"graphgen": build_graphgen, "coop": build_coop, "all": build_all}[w]()
