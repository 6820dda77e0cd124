"""Compile the C oracle (test infrastructure) with gcc into oracle/liboracle.so."""
from __future__ import annotations

import os
import subprocess

ORACLE_DIR = os.path.dirname(os.path.abspath(__file__))
ORACLE_SO = os.path.join(ORACLE_DIR, "liboracle.so")


def build_oracle() -> str:
    tmp = ORACLE_SO + ".tmp"
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-std=c11",
           os.path.join(ORACLE_DIR, "oracle.c"), "-o", tmp]
    print("+", " ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, ORACLE_SO)
    return ORACLE_SO


if __name__ == "__main__":
    build_oracle()
