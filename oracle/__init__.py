"""CPU oracle for the cooperative graph-traversal path.

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. The GPU library
never calls it, and the two share no code (only the seeded input generators
in ``paper_1707_01989_amd.graphgen`` feed both).

The arithmetic lives in ``oracle.c`` (plain C, one obviously-correct textbook
algorithm per function); this module only marshals numpy arrays.

Functions (all results are integer and unique):
  bfs(g, src)         -> uint32[n] levels, 0xFFFFFFFF = unreached
  sssp(g, src)        -> int32[n] distances, INT32_MAX = unreached
  color(g, prio_seed) -> uint32[n] greedy colours in decreasing key order
  mis(g, prio_seed)   -> uint8[n] greedy maximal independent set, same order
  cc(g)               -> uint32[n] connected-component labels, each the smallest
                         vertex id of its component
  priority_order(n, prio_seed) -> vertices by decreasing key
  octree(x, y, z, cap) -> (uint32[n, 4] points in final order {x, y, z, index},
                           uint32[k, 5] leaves {first, end, depth, code_lo, code_hi})
  splitmix64(x)       -> SplitMix64 output for state x

All-core CPU baselines (``cpu_parallel.c``, OpenMP; not the oracle, pinned to
it by tests, timed by the benchmark beside it):
  bfs_parallel(g, src, threads=0)  -> (uint32[n] levels, threads used)
  sssp_parallel(g, src, threads=0) -> (int32[n] distances, threads used)

The cooperative-scheduling semantics model lives in ``oracle.coop_model``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

UNREACHED_LEVEL = 0xFFFFFFFF
UNREACHED_DIST = 0x7FFFFFFF

_lib = None
_par = None


class OracleError(RuntimeError):
    pass


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_build.ORACLE_SO):
        _build.build_oracle()
    lib = ctypes.CDLL(_build.ORACLE_SO)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    i32p = ctypes.POINTER(ctypes.c_int32)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    lib.oracle_splitmix64.restype = ctypes.c_uint64
    lib.oracle_splitmix64.argtypes = [ctypes.c_uint64]
    lib.oracle_bfs.restype = ctypes.c_int
    lib.oracle_bfs.argtypes = [ctypes.c_uint32, u32p, u32p, ctypes.c_uint32, u32p]
    lib.oracle_sssp.restype = ctypes.c_int
    lib.oracle_sssp.argtypes = [ctypes.c_uint32, u32p, u32p, u32p, ctypes.c_uint32, i32p]
    lib.oracle_color.restype = ctypes.c_int
    lib.oracle_color.argtypes = [ctypes.c_uint32, u32p, u32p, ctypes.c_uint64, u32p]
    lib.oracle_mis.restype = ctypes.c_int
    lib.oracle_mis.argtypes = [ctypes.c_uint32, u32p, u32p, ctypes.c_uint64, u8p]
    lib.oracle_cc.restype = ctypes.c_int
    lib.oracle_cc.argtypes = [ctypes.c_uint32, u32p, u32p, u32p]
    lib.oracle_octree.restype = ctypes.c_int
    lib.oracle_octree.argtypes = [ctypes.c_uint32, u32p, u32p, u32p, ctypes.c_uint32, u32p, u32p,
                                  ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)]
    lib.oracle_priority_order.restype = ctypes.c_int
    lib.oracle_priority_order.argtypes = [ctypes.c_uint32, ctypes.c_uint64, u32p]
    _lib = lib
    return lib


def _load_parallel():
    global _par
    if _par is not None:
        return _par
    if not os.path.exists(_build.PARALLEL_SO):
        _build.build_parallel()
    lib = ctypes.CDLL(_build.PARALLEL_SO)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.cpu_bfs_par.restype = ctypes.c_int
    lib.cpu_bfs_par.argtypes = [ctypes.c_uint32, u32p, u32p, ctypes.c_uint32, u32p, ctypes.c_int]
    lib.cpu_sssp_par.restype = ctypes.c_int
    lib.cpu_sssp_par.argtypes = [ctypes.c_uint32, u32p, u32p, u32p, ctypes.c_uint32, i32p, ctypes.c_int]
    _par = lib
    return lib


def _ptr(a: np.ndarray, ct):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _u32(a):
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return a, _ptr(a, ctypes.c_uint32)


def splitmix64(x: int) -> int:
    return int(_load().oracle_splitmix64(ctypes.c_uint64(x & (2**64 - 1))))


def bfs(g, src: int) -> np.ndarray:
    rp, prp = _u32(g.row_ptr)
    col, pcol = _u32(g.col)
    out = np.empty(g.n, dtype=np.uint32)
    rc = _load().oracle_bfs(g.n, prp, pcol, src, _ptr(out, ctypes.c_uint32))
    if rc != 0:
        raise OracleError(f"oracle_bfs failed ({rc})")
    return out


def sssp(g, src: int) -> np.ndarray:
    if g.w is None:
        raise OracleError("sssp needs weights")
    rp, prp = _u32(g.row_ptr)
    col, pcol = _u32(g.col)
    w, pw = _u32(g.w)
    out = np.empty(g.n, dtype=np.int32)
    rc = _load().oracle_sssp(g.n, prp, pcol, pw, src, _ptr(out, ctypes.c_int32))
    if rc == -6:
        raise OverflowError("shortest-path distance exceeds int32")
    if rc != 0:
        raise OracleError(f"oracle_sssp failed ({rc})")
    return out


def color(g, prio_seed: int) -> np.ndarray:
    rp, prp = _u32(g.row_ptr)
    col, pcol = _u32(g.col)
    out = np.empty(g.n, dtype=np.uint32)
    rc = _load().oracle_color(g.n, prp, pcol, prio_seed & (2**64 - 1), _ptr(out, ctypes.c_uint32))
    if rc != 0:
        raise OracleError(f"oracle_color failed ({rc})")
    return out


def mis(g, prio_seed: int) -> np.ndarray:
    rp, prp = _u32(g.row_ptr)
    col, pcol = _u32(g.col)
    out = np.empty(g.n, dtype=np.uint8)
    rc = _load().oracle_mis(g.n, prp, pcol, prio_seed & (2**64 - 1), _ptr(out, ctypes.c_uint8))
    if rc != 0:
        raise OracleError(f"oracle_mis failed ({rc})")
    return out


def cc(g) -> np.ndarray:
    rp, prp = _u32(g.row_ptr)
    col, pcol = _u32(g.col)
    out = np.empty(g.n, dtype=np.uint32)
    rc = _load().oracle_cc(g.n, prp, pcol, _ptr(out, ctypes.c_uint32))
    if rc != 0:
        raise OracleError(f"oracle_cc failed ({rc})")
    return out


def priority_order(n: int, prio_seed: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint32)
    rc = _load().oracle_priority_order(n, prio_seed & (2**64 - 1), _ptr(out, ctypes.c_uint32))
    if rc != 0:
        raise OracleError("oracle_priority_order failed")
    return out


def octree(x, y, z, cap: int) -> tuple[np.ndarray, np.ndarray]:
    """Octree of integer points (see oracle_octree): the points in final
    order as rows {x, y, z, original index}, and the leaves as rows
    {first, end, depth, code_lo, code_hi} in order."""
    x, px = _u32(x)
    y, py = _u32(y)
    z, pz = _u32(z)
    n = len(x)
    out = np.zeros((n, 4), dtype=np.uint32)
    max_leaves = max(1, n)
    leaves = np.zeros((max_leaves, 5), dtype=np.uint32)
    nl = ctypes.c_uint64()
    rc = _load().oracle_octree(n, px, py, pz, cap, _ptr(out, ctypes.c_uint32), _ptr(leaves, ctypes.c_uint32),
                               max_leaves, ctypes.byref(nl))
    if rc != 0:
        raise OracleError(f"oracle_octree failed ({rc})")
    return out, leaves[: nl.value].copy()


def bfs_parallel(g, src: int, threads: int = 0) -> tuple[np.ndarray, int]:
    """All-core level-synchronous BFS (OpenMP); threads = 0: the OpenMP default."""
    rp, prp = _u32(g.row_ptr)
    col, pcol = _u32(g.col)
    out = np.empty(g.n, dtype=np.uint32)
    rc = _load_parallel().cpu_bfs_par(g.n, prp, pcol, src, _ptr(out, ctypes.c_uint32), threads)
    if rc <= 0:
        raise OracleError(f"cpu_bfs_par failed ({rc})")
    return out, rc


def sssp_parallel(g, src: int, threads: int = 0) -> tuple[np.ndarray, int]:
    """All-core frontier Bellman-Ford (OpenMP); threads = 0: the OpenMP default."""
    if g.w is None:
        raise OracleError("sssp needs weights")
    rp, prp = _u32(g.row_ptr)
    col, pcol = _u32(g.col)
    w, pw = _u32(g.w)
    out = np.empty(g.n, dtype=np.int32)
    rc = _load_parallel().cpu_sssp_par(g.n, prp, pcol, pw, src, _ptr(out, ctypes.c_int32), threads)
    if rc == -6:
        raise OverflowError("shortest-path distance exceeds int32")
    if rc <= 0:
        raise OracleError(f"cpu_sssp_par failed ({rc})")
    return out, rc
