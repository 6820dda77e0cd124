"""Seeded synthetic graph inputs (shared by the library's callers and the tests).

This module only *generates inputs*: CSR graphs, per-edge weights and source
vertices, from counter-based SplitMix64 draws (implemented in
``csrc/graphgen.c``). It holds none of the traversal arithmetic.

Conventions (the paper does not fix a graph layout):
  * CSR with ``row_ptr`` (uint32, n+1) and ``col`` (uint32, arcs);
  * symmetric: every undirected edge is stored as two arcs;
  * no self loops, no duplicate edges, adjacency lists sorted ascending;
  * weights (uint32) belong to the undirected edge, so both arcs agree.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from . import build as _build

_lib = None

STREAM_ER, STREAM_RMAT, STREAM_PERM, STREAM_W, STREAM_MISC = 1, 2, 3, 4, 5


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_build.GRAPHGEN_SO):
        _build.build_graphgen()
    lib = ctypes.CDLL(_build.GRAPHGEN_SO)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    lib.gg_splitmix64.restype = ctypes.c_uint64
    lib.gg_splitmix64.argtypes = [ctypes.c_uint64]
    lib.gg_rand.restype = ctypes.c_uint64
    lib.gg_rand.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64]
    lib.gg_uniform.restype = ctypes.c_uint64
    lib.gg_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                               ctypes.c_uint64, ctypes.c_uint64]
    lib.gg_real.restype = ctypes.c_double
    lib.gg_real.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64]
    lib.gg_er_edges.restype = ctypes.c_int64
    lib.gg_er_edges.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, u32p, u32p]
    lib.gg_grid_edges.restype = ctypes.c_int64
    lib.gg_grid_edges.argtypes = [ctypes.c_uint32, ctypes.c_uint32, u32p, u32p]
    lib.gg_rmat_edges.restype = ctypes.c_int64
    lib.gg_rmat_edges.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_uint64, u32p, u32p]
    lib.gg_canonical_edges.restype = ctypes.c_int64
    lib.gg_canonical_edges.argtypes = [ctypes.c_uint64, u32p, u32p]
    lib.gg_csr.restype = ctypes.c_int
    lib.gg_csr.argtypes = [ctypes.c_uint32, ctypes.c_uint64, u32p, u32p, u32p, u32p]
    lib.gg_weights.restype = ctypes.c_int
    lib.gg_weights.argtypes = [ctypes.c_uint32, u32p, u32p, ctypes.c_uint64,
                               ctypes.c_uint32, ctypes.c_uint32, u32p]
    lib.gg_points.restype = ctypes.c_int
    lib.gg_points.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32, u32p, u32p, u32p]
    lib.gg_sources.restype = ctypes.c_int64
    lib.gg_sources.argtypes = [ctypes.c_uint32, u32p, ctypes.c_uint64, ctypes.c_uint32, u32p]
    _lib = lib
    return lib


def _p(a: np.ndarray):
    assert a.dtype == np.uint32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


@dataclass
class Graph:
    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    w: Optional[np.ndarray] = None
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def arcs(self) -> int:
        return int(self.col.shape[0])

    @property
    def edges(self) -> int:
        return self.arcs // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))


# ------------------------------------------------------------------ draws

def splitmix64(x: int) -> int:
    return int(_load().gg_splitmix64(ctypes.c_uint64(x & (2**64 - 1))))


def rand(seed: int, stream: int, i: int) -> int:
    return int(_load().gg_rand(seed & (2**64 - 1), stream, i))


def uniform(seed: int, stream: int, i: int, lo: int, hi: int) -> int:
    return int(_load().gg_uniform(seed & (2**64 - 1), stream, i, lo, hi))


def real(seed: int, stream: int, i: int) -> float:
    return float(_load().gg_real(seed & (2**64 - 1), stream, i))


# ---------------------------------------------------------------- packing

def _csr_from_sorted(n: int, eu: np.ndarray, ev: np.ndarray, name: str, **meta) -> Graph:
    m = int(eu.shape[0])
    row_ptr = np.zeros(n + 1, dtype=np.uint32)
    col = np.zeros(2 * m, dtype=np.uint32)
    rc = _load().gg_csr(n, m, _p(eu), _p(ev), _p(row_ptr), _p(col))
    if rc != 0:
        raise ValueError(f"gg_csr failed ({rc})")
    return Graph(n=n, row_ptr=row_ptr, col=col, name=name, meta=dict(meta))


def from_edges(n: int, u, v, name: str = "edges") -> Graph:
    """Canonicalise an arbitrary edge list (drop loops/duplicates) into CSR."""
    eu = np.ascontiguousarray(np.asarray(u, dtype=np.uint32)).copy()
    ev = np.ascontiguousarray(np.asarray(v, dtype=np.uint32)).copy()
    if eu.size and (eu.max() >= n or ev.max() >= n):
        raise ValueError("endpoint out of range")
    m = _load().gg_canonical_edges(eu.size, _p(eu), _p(ev))
    return _csr_from_sorted(n, eu[:m].copy(), ev[:m].copy(), name)


def er(n: int, avg_deg: float, seed: int) -> Graph:
    """Erdos-Renyi G(n, m) with m = floor(n * avg_deg / 2 + 0.5) distinct edges."""
    m = int(np.floor(n * avg_deg / 2.0 + 0.5))
    eu = np.zeros(max(m, 1), dtype=np.uint32)
    ev = np.zeros(max(m, 1), dtype=np.uint32)
    got = _load().gg_er_edges(n, m, seed & (2**64 - 1), _p(eu), _p(ev))
    if got != m:
        raise ValueError(f"G(n={n}, m={m}) impossible")
    return _csr_from_sorted(n, eu[:m], ev[:m], f"er{n}_d{avg_deg}_s{seed}",
                            family="er", avg_deg=avg_deg, seed=seed)


def batch_sizes(count: int = 512, seed0: int = 1000, log2_lo: float = 10.0, log2_hi: float = 18.0,
                deg_lo: float = 4.0, deg_hi: float = 32.0) -> list[tuple[int, float, int]]:
    """(n_i, d_i, seed_i) of a batch of ER instances: instance i uses seed
    seed0 + i; n_i = floor(2^U(log2_lo, log2_hi)) (log-uniform vertex
    count), d_i = U(deg_lo, deg_hi) (average degree), both drawn from
    stream 11 of that seed."""
    out = []
    for i in range(count):
        s = seed0 + i
        n = int(np.floor(2.0 ** (log2_lo + (log2_hi - log2_lo) * real(s, 11, 0))))
        d = deg_lo + (deg_hi - deg_lo) * real(s, 11, 1)
        out.append((n, d, s))
    return out


def er_batch(count: int = 512, seed0: int = 1000, workers: int = 8, **kw) -> list[Graph]:
    """The ER instances of batch_sizes(), generated in parallel threads (the
    C generator releases the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor
    sizes = batch_sizes(count, seed0, **kw)
    with ThreadPoolExecutor(max_workers=max(1, workers)) as ex:
        return list(ex.map(lambda t: er(t[0], t[1], t[2]), sizes))


def grid(R: int, C: int) -> Graph:
    m = R * (C - 1) + (R - 1) * C
    eu = np.zeros(max(m, 1), dtype=np.uint32)
    ev = np.zeros(max(m, 1), dtype=np.uint32)
    got = _load().gg_grid_edges(R, C, _p(eu), _p(ev))
    assert got == m
    return _csr_from_sorted(R * C, eu[:m], ev[:m], f"grid{R}x{C}", family="grid", R=R, C=C)


def rmat(scale: int, edgefactor: int = 16, seed: int = 3,
         a: float = 0.57, b: float = 0.19, c: float = 0.19) -> Graph:
    n = 1 << scale
    draws = edgefactor * n
    eu = np.zeros(draws, dtype=np.uint32)
    ev = np.zeros(draws, dtype=np.uint32)
    got = _load().gg_rmat_edges(scale, edgefactor, a, b, c, seed & (2**64 - 1), _p(eu), _p(ev))
    if got < 0:
        raise ValueError("bad R-MAT parameters")
    eu = eu[:got].copy()
    ev = ev[:got].copy()
    return _csr_from_sorted(n, eu, ev, f"rmat{scale}_ef{edgefactor}_s{seed}", family="rmat",
                            scale=scale, edgefactor=edgefactor, seed=seed)


def add_weights(g: Graph, seed: int, lo: int, hi: int) -> Graph:
    w = np.zeros(g.arcs, dtype=np.uint32)
    rc = _load().gg_weights(g.n, _p(g.row_ptr), _p(g.col), seed & (2**64 - 1), lo, hi, _p(w))
    if rc != 0:
        raise ValueError("weights need n <= 2^24 and lo <= hi")
    g.w = w
    g.meta.update(w_seed=seed, w_lo=lo, w_hi=hi)
    return g


def constant_weights(g: Graph, value: int) -> Graph:
    g.w = np.full(g.arcs, value, dtype=np.uint32)
    return g


def sources(g: Graph, seed: int, k: int) -> np.ndarray:
    out = np.zeros(max(k, 1), dtype=np.uint32)
    got = _load().gg_sources(g.n, _p(g.row_ptr), seed & (2**64 - 1), k, _p(out))
    if got == 0 and k > 0:
        raise ValueError("graph has no vertex of degree >= 1")
    return out[:k]


# ------------------------------------------------- small closed-form graphs

def path(n: int) -> Graph:
    i = np.arange(max(n - 1, 0), dtype=np.uint32)
    return from_edges(n, i, i + 1, f"path{n}")


def cycle(n: int) -> Graph:
    i = np.arange(n, dtype=np.uint32)
    return from_edges(n, i, (i + 1) % n, f"cycle{n}")


def star(n: int) -> Graph:
    leaves = np.arange(1, n, dtype=np.uint32)
    return from_edges(n, np.zeros_like(leaves), leaves, f"star{n}")


def complete(n: int) -> Graph:
    u, v = np.triu_indices(n, 1)
    return from_edges(n, u, v, f"K{n}")


def complete_bipartite(a: int, b: int) -> Graph:
    u, v = np.meshgrid(np.arange(a), np.arange(a, a + b), indexing="ij")
    return from_edges(a + b, u.ravel(), v.ravel(), f"K{a},{b}")


def binary_tree(n: int) -> Graph:
    """Complete binary tree in heap order: parent of i is (i-1)//2."""
    i = np.arange(1, n, dtype=np.uint32)
    return from_edges(n, (i - 1) // 2, i, f"bintree{n}")


def empty(n: int) -> Graph:
    return Graph(n=n, row_ptr=np.zeros(n + 1, dtype=np.uint32),
                 col=np.zeros(0, dtype=np.uint32), name=f"empty{n}")


def disjoint_union(g1: Graph, g2: Graph) -> Graph:
    rp = np.concatenate([g1.row_ptr[:-1], g2.row_ptr + np.uint32(g1.arcs)]).astype(np.uint32)
    col = np.concatenate([g1.col, g2.col + np.uint32(g1.n)]).astype(np.uint32)
    w = None
    if g1.w is not None and g2.w is not None:
        w = np.concatenate([g1.w, g2.w]).astype(np.uint32)
    return Graph(n=g1.n + g2.n, row_ptr=rp, col=col, w=w, name=f"{g1.name}+{g2.name}")


# ----------------------------------------------------------------- points

POINT_BITS = 21          # coordinates in [0, 2^21) per axis


def points(n: int, seed: int, kind: str = "uniform") -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """n seeded points (x, y, z uint32 arrays in [0, 2^21)): "uniform", or
    "clustered" (16 seeded centres, bell-shaped spread of about 1% of the
    side), for the work-stealing octree."""
    k = {"uniform": 0, "clustered": 1}[kind]
    x = np.zeros(n, dtype=np.uint32)
    y = np.zeros(n, dtype=np.uint32)
    z = np.zeros(n, dtype=np.uint32)
    if n:
        rc = _load().gg_points(n, seed & (2**64 - 1), k, _p(x), _p(y), _p(z))
        if rc != 0:
            raise ValueError("gg_points failed")
    return x, y, z
