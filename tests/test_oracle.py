"""Pins for the CPU oracle, checked against things other than itself:
closed forms, brute force (Floyd-Warshall, full Bellman-Ford passes),
library routines (scipy.sparse.csgraph), and local characterisations that
determine the result uniquely."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse import csgraph

import oracle
from oracle import UNREACHED_DIST, UNREACHED_LEVEL

GAMMA = 0x9E3779B97F4A7C15
MASK = 2**64 - 1


# ------------------------------------------------------------- helpers

def to_scipy(g, weighted=False):
    data = g.w.astype(np.float64) if weighted else np.ones(g.arcs)
    return sp.csr_matrix((data, g.col.astype(np.int64), g.row_ptr.astype(np.int64)),
                         shape=(g.n, g.n))


def floyd_warshall(g, weighted):
    n = g.n
    D = np.full((n, n), np.inf)
    np.fill_diagonal(D, 0)
    for v in range(n):
        for e in range(g.row_ptr[v], g.row_ptr[v + 1]):
            D[v, g.col[e]] = min(D[v, g.col[e]], g.w[e] if weighted else 1)
    for k in range(n):
        D = np.minimum(D, D[:, k:k + 1] + D[k:k + 1, :])
    return D


def as_levels(row):
    return np.where(np.isinf(row), UNREACHED_LEVEL, row).astype(np.uint32)


def as_dists(row):
    return np.where(np.isinf(row), UNREACHED_DIST, row).astype(np.int32)


def keys(gg, n, prio_seed):
    """h(v) = output v of SplitMix64 started at prio_seed, computed through the
    generator module's own SplitMix64 (separate code from the oracle's)."""
    return [gg.splitmix64((prio_seed + v * GAMMA) & MASK) for v in range(n)]


def higher(kv, u, v):
    return (kv[u], u) > (kv[v], v)


# ----------------------------------------------------------------- BFS

def test_bfs_closed_forms(gg):
    n = 9
    assert np.array_equal(oracle.bfs(gg.path(n), 0), np.arange(n))
    assert np.array_equal(oracle.bfs(gg.path(n), 4), np.abs(np.arange(n) - 4))
    i = np.arange(n)
    assert np.array_equal(oracle.bfs(gg.cycle(n), 2), np.minimum(np.abs(i - 2), n - np.abs(i - 2)))
    lk = oracle.bfs(gg.complete(7), 3)
    assert lk[3] == 0 and np.all(np.delete(lk, 3) == 1)
    ls = oracle.bfs(gg.star(8), 5)
    assert ls[5] == 0 and ls[0] == 1 and np.all(np.delete(ls, [0, 5]) == 2)
    lt = oracle.bfs(gg.binary_tree(31), 0)
    assert np.array_equal(lt, np.floor(np.log2(np.arange(31) + 1)).astype(np.uint32))
    R, C = 6, 9
    lg = oracle.bfs(gg.grid(R, C), 0)
    rr, cc = np.divmod(np.arange(R * C), C)
    assert np.array_equal(lg, rr + cc)


def test_bfs_unreached_sentinel(gg):
    g = gg.disjoint_union(gg.path(4), gg.cycle(5))
    lv = oracle.bfs(g, 1)
    assert np.array_equal(lv[:4], [1, 0, 1, 2])
    assert np.all(lv[4:] == UNREACHED_LEVEL)
    lone = oracle.bfs(gg.empty(3), 2)
    assert list(lone) == [UNREACHED_LEVEL, UNREACHED_LEVEL, 0]


@pytest.mark.parametrize("seed", range(6))
def test_bfs_brute_force(gg, seed):
    g = gg.er(40 + seed * 4, 2.5, 100 + seed)    # sparse enough to be disconnected
    D = floyd_warshall(g, weighted=False)
    for s in (0, g.n // 2, g.n - 1):
        assert np.array_equal(oracle.bfs(g, s), as_levels(D[s]))


@pytest.mark.parametrize("make", ["er", "rmat", "grid"])
def test_bfs_vs_scipy_and_invariants(gg, make):
    g = {"er": lambda: gg.er(20000, 6, 4), "rmat": lambda: gg.rmat(13, 16, seed=8),
         "grid": lambda: gg.grid(60, 70)}[make]()
    src = int(gg.sources(g, 1, 1)[0])
    lv = oracle.bfs(g, src)
    ref = csgraph.shortest_path(to_scipy(g), unweighted=True, indices=src)
    assert np.array_equal(lv, as_levels(ref))
    reached = lv != UNREACHED_LEVEL
    srcs = np.repeat(np.arange(g.n), g.degrees())
    both = reached[srcs] & reached[g.col]
    diff = lv[srcs][both].astype(np.int64) - lv[g.col][both].astype(np.int64)
    assert np.all(np.abs(diff) <= 1)
    # every reached vertex but the source has a neighbour one level closer
    has_parent = np.zeros(g.n, bool)
    ok = both & (lv[g.col].astype(np.int64) == lv[srcs].astype(np.int64) - 1)
    has_parent[srcs[ok]] = True
    assert np.all(has_parent[reached] | (np.arange(g.n)[reached] == src))
    # reached set is exactly the connected component of the source
    _, comp = csgraph.connected_components(to_scipy(g), directed=False)
    assert np.array_equal(reached, comp == comp[src])


def test_bfs_bad_source(gg):
    with pytest.raises(oracle.OracleError):
        oracle.bfs(gg.path(3), 3)


# ---------------------------------------------------------------- SSSP

def test_sssp_closed_forms(gg):
    # unit weights: distances are BFS levels
    g = gg.constant_weights(gg.er(500, 5, 3), 1)
    bfs = oracle.bfs(g, 7).astype(np.int64)
    d = oracle.sssp(g, 7)
    assert np.array_equal(np.where(bfs == UNREACHED_LEVEL, UNREACHED_DIST, bfs), d)
    # constant weight on a grid from the corner: w * (r + c)
    R, C, w = 7, 11, 13
    g = gg.constant_weights(gg.grid(R, C), w)
    rr, cc = np.divmod(np.arange(R * C), C)
    assert np.array_equal(oracle.sssp(g, 0), w * (rr + cc))
    # path: prefix sums of the edge weights
    g = gg.add_weights(gg.path(12), 5, 1, 1000)
    ew = np.array([g.w[g.row_ptr[i]:g.row_ptr[i + 1]][g.col[g.row_ptr[i]:g.row_ptr[i + 1]] == i + 1][0]
                   for i in range(11)], dtype=np.int64)
    assert np.array_equal(oracle.sssp(g, 0), np.concatenate([[0], np.cumsum(ew)]))


@pytest.mark.parametrize("seed", range(6))
def test_sssp_brute_force(gg, seed):
    g = gg.add_weights(gg.er(36 + seed * 5, 3.0, 200 + seed), seed, 1, 1000)
    D = floyd_warshall(g, weighted=True)
    for s in (0, g.n // 3, g.n - 1):
        assert np.array_equal(oracle.sssp(g, s), as_dists(D[s]))


def bellman_ford(g, s):
    """n-1 full passes of edge relaxation (vectorised), 64-bit."""
    d = np.full(g.n, np.iinfo(np.int64).max // 4, dtype=np.int64)
    d[s] = 0
    srcs = np.repeat(np.arange(g.n), g.degrees())
    for _ in range(g.n - 1):
        cand = d[srcs] + g.w.astype(np.int64)
        nd = d.copy()
        np.minimum.at(nd, g.col, cand)
        if np.array_equal(nd, d):
            break
        d = nd
    return np.where(d >= np.iinfo(np.int64).max // 8, UNREACHED_DIST, d).astype(np.int32)


@pytest.mark.parametrize("make", ["grid", "rmat", "er"])
def test_sssp_vs_bellman_ford_scipy_and_invariants(gg, make):
    g = {"grid": lambda: gg.add_weights(gg.grid(30, 40), 2, 1, 1000),
         "rmat": lambda: gg.add_weights(gg.rmat(11, 16, seed=4), 4, 1, 255),
         "er": lambda: gg.add_weights(gg.er(3000, 4, 9), 9, 1, 1000)}[make]()
    src = int(gg.sources(g, 6, 1)[0])
    d = oracle.sssp(g, src)
    assert np.array_equal(d, bellman_ford(g, src))
    ref = csgraph.dijkstra(to_scipy(g, weighted=True), indices=src)
    assert np.array_equal(d, as_dists(ref))
    reached = d != UNREACHED_DIST
    srcs = np.repeat(np.arange(g.n), g.degrees())
    both = reached[srcs] & reached[g.col]
    du, dv = d[srcs].astype(np.int64), d[g.col].astype(np.int64)
    assert np.all(dv[both] <= du[both] + g.w[both])                # feasible
    tight = np.zeros(g.n, bool)
    tight[g.col[both & (dv == du + g.w)]] = True
    assert np.all(tight[reached] | (np.arange(g.n)[reached] == src))  # every vertex has a tight arc
    assert np.array_equal(reached, oracle.bfs(g, src) != UNREACHED_LEVEL)


def test_sssp_overflow(gg):
    g = gg.constant_weights(gg.path(5), 1_000_000_000)
    with pytest.raises(OverflowError):
        oracle.sssp(g, 0)


# ----------------------------------------------------------- colouring

def mex(values):
    s = set(values)
    c = 0
    while c in s:
        c += 1
    return c


def verify_colouring(g, colour, kv):
    """colour[v] == mex over higher-key neighbours for every v. By induction
    over decreasing key this characterises the greedy colouring uniquely."""
    for v in range(g.n):
        nb = g.col[g.row_ptr[v]:g.row_ptr[v + 1]]
        hi = [int(colour[u]) for u in nb if higher(kv, int(u), v)]
        if int(colour[v]) != mex(hi):
            return False
    return True


def brute_greedy_colour(g, kv):
    order = sorted(range(g.n), key=lambda v: (kv[v], v), reverse=True)
    colour = [None] * g.n
    for v in order:
        colour[v] = mex(colour[int(u)] for u in g.col[g.row_ptr[v]:g.row_ptr[v + 1]]
                        if colour[int(u)] is not None)
    return np.array(colour, dtype=np.uint32)


@pytest.mark.parametrize("seed", [0, 1, 77])
def test_color_local_characterisation(gg, seed):
    g = gg.er(1500, 10, 30 + seed)
    kv = keys(gg, g.n, seed)
    col = oracle.color(g, seed)
    assert verify_colouring(g, col, kv)
    srcs = np.repeat(np.arange(g.n), g.degrees())
    assert not np.any(col[srcs] == col[g.col])                      # proper
    assert np.all(col <= g.degrees())


def test_color_brute_force(gg):
    for seed in range(4):
        g = gg.er(60, 6, 300 + seed)
        kv = keys(gg, g.n, seed)
        assert np.array_equal(oracle.color(g, seed), brute_greedy_colour(g, kv))


def test_color_closed_forms(gg):
    seed = 12345
    n = 9
    kv = keys(gg, n, seed)
    order = sorted(range(n), key=lambda v: (kv[v], v), reverse=True)
    col = oracle.color(gg.complete(n), seed)
    assert [int(col[v]) for v in order] == list(range(n))
    assert np.all(oracle.color(gg.empty(6), seed) == 0)
    a, b = 4, 5
    kv = keys(gg, a + b, seed)
    top = max(range(a + b), key=lambda v: (kv[v], v))
    col = oracle.color(gg.complete_bipartite(a, b), seed)
    side_top = np.arange(a + b) < a if top < a else np.arange(a + b) >= a
    assert np.all(col[side_top] == 0) and np.all(col[~side_top] == 1)


def test_color_verifier_catches_planted_error(gg):
    g = gg.er(300, 8, 5)
    kv = keys(gg, g.n, 3)
    col = oracle.color(g, 3).copy()
    col[17] += 1
    assert not verify_colouring(g, col, kv)


def test_priority_order_matches_keys(gg):
    n, seed = 500, 99
    kv = keys(gg, n, seed)
    exp = sorted(range(n), key=lambda v: (kv[v], v), reverse=True)
    assert list(oracle.priority_order(n, seed)) == exp


# ----------------------------------------------------------------- MIS

def verify_mis(g, ins, kv):
    """v in I <=> no higher-key neighbour is in I (characterises the greedy
    MIS in decreasing key order)."""
    for v in range(g.n):
        nb = g.col[g.row_ptr[v]:g.row_ptr[v + 1]]
        blocked = any(ins[u] for u in nb if higher(kv, int(u), v))
        if bool(ins[v]) == blocked:
            return False
    return True


@pytest.mark.parametrize("seed", [0, 5])
def test_mis_local_characterisation(gg, seed):
    g = gg.rmat(11, 8, seed=seed + 1)
    kv = keys(gg, g.n, seed)
    ins = oracle.mis(g, seed)
    assert verify_mis(g, ins, kv)
    srcs = np.repeat(np.arange(g.n), g.degrees())
    assert not np.any(ins[srcs] & ins[g.col])                          # independent
    dominated = np.zeros(g.n, bool)
    dominated[g.col[ins[srcs] == 1]] = True
    assert np.all(ins.astype(bool) | dominated)                        # maximal


def test_mis_closed_forms(gg):
    seed = 4242
    n = 8
    kv = keys(gg, n, seed)
    top = max(range(n), key=lambda v: (kv[v], v))
    ins = oracle.mis(gg.complete(n), seed)
    assert list(np.nonzero(ins)[0]) == [top]
    assert np.all(oracle.mis(gg.empty(5), seed) == 1)
    ins = oracle.mis(gg.star(n), seed)
    if top == 0:
        assert list(np.nonzero(ins)[0]) == [0]
    else:
        assert ins[0] == 0 and np.all(ins[1:] == 1)


def test_mis_verifier_catches_planted_error(gg):
    g = gg.er(300, 8, 6)
    kv = keys(gg, g.n, 1)
    ins = oracle.mis(g, 1).copy()
    v = int(np.nonzero(ins)[0][0])
    ins[v] = 0
    assert not verify_mis(g, ins, kv)


# --------------------------------------------------- connected components

def cc_min_labels_scipy(g):
    """Smallest vertex id of every vertex's component, from scipy's
    connected_components (its own component numbering, mapped to minima)."""
    k, comp = csgraph.connected_components(to_scipy(g), directed=False)
    mins = np.full(k, np.iinfo(np.int64).max)
    np.minimum.at(mins, comp, np.arange(g.n))
    return mins[comp].astype(np.uint32)


@pytest.mark.parametrize("make", [
    lambda gg: gg.er(2000, 1.5, 4),           # many components near the ER threshold
    lambda gg: gg.er(3000, 8, 5),
    lambda gg: gg.rmat(12, 8, seed=6),        # isolated vertices and one giant component
    lambda gg: gg.grid(30, 40),
    lambda gg: gg.disjoint_union(gg.disjoint_union(gg.path(50), gg.empty(9)), gg.star(30)),
])
def test_cc_vs_scipy(gg, make):
    g = make(gg)
    assert np.array_equal(oracle.cc(g), cc_min_labels_scipy(g))


def test_cc_closed_forms(gg):
    assert np.array_equal(oracle.cc(gg.path(100)), np.zeros(100, np.uint32))
    assert np.array_equal(oracle.cc(gg.empty(17)), np.arange(17, dtype=np.uint32))
    u = gg.disjoint_union(gg.complete(5), gg.disjoint_union(gg.empty(3), gg.path(4)))
    assert list(oracle.cc(u)) == [0] * 5 + [5, 6, 7] + [8] * 4


def test_cc_characterisation(gg):
    """The labels are the fixed point of minimum-label propagation that is
    also minimal: every arc joins equal labels, every label is a vertex of
    its own class and the smallest one, and classes are connected (the BFS
    levels from the label reach exactly the class)."""
    g = gg.er(1500, 2.0, 9)
    lab = oracle.cc(g)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr.astype(np.int64)))
    assert np.all(lab[src] == lab[g.col])
    assert np.all(lab <= np.arange(g.n))
    assert np.all(lab[lab] == lab)
    for r in np.unique(lab)[:50]:
        reach = oracle.bfs(g, int(r)) != UNREACHED_LEVEL
        assert np.array_equal(reach, lab == r)


def test_cc_checks_catch_planted_error(gg):
    g = gg.er(800, 3.0, 2)
    lab = oracle.cc(g).copy()
    v = int(np.nonzero(lab != np.arange(g.n))[0][0])
    lab[v] = v                                  # split a vertex off its component
    assert not np.array_equal(lab, cc_min_labels_scipy(g))
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr.astype(np.int64)))
    assert not np.all(lab[src] == lab[g.col])
