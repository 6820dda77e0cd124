"""Compile the C oracle (test infrastructure) with gcc into oracle/liboracle.so, and the
all-core CPU baselines into oracle/libcpu_parallel.so."""
from __future__ import annotations

import os
import subprocess

ORACLE_DIR = os.path.dirname(os.path.abspath(__file__))
ORACLE_SO = os.path.join(ORACLE_DIR, "liboracle.so")
PARALLEL_SO = os.path.join(ORACLE_DIR, "libcpu_parallel.so")


def build_oracle() -> str:
    tmp = ORACLE_SO + ".tmp"
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-std=c11",
           os.path.join(ORACLE_DIR, "oracle.c"), "-o", tmp]
    print("+", " ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, ORACLE_SO)
    build_parallel()
    return ORACLE_SO


def build_parallel() -> str:
    """The all-core CPU baselines (OpenMP), pinned to the oracle by tests."""
    tmp = PARALLEL_SO + ".tmp"
    cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           os.path.join(ORACLE_DIR, "cpu_parallel.c"), "-o", tmp]
    print("+", " ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, PARALLEL_SO)
    return PARALLEL_SO


if __name__ == "__main__":
    build_oracle()
