"""Seeded input generators: determinism, structure and the SplitMix64 pins."""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64.txt")


def _golden():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        a, b = line.split()
        rows.append((int(a, 16), int(b, 16)))
    return rows


def test_splitmix64_reference_outputs(gg):
    for state, out in _golden():
        assert gg.splitmix64(state) == out


def check_simple_symmetric(g):
    rp = g.row_ptr.astype(np.int64)
    assert rp[0] == 0 and rp[-1] == g.arcs
    assert np.all(np.diff(rp) >= 0)
    src = np.repeat(np.arange(g.n), np.diff(rp))
    col = g.col.astype(np.int64)
    assert np.all(col < g.n)
    assert not np.any(src == col), "self loop"
    # sorted strictly ascending inside each row => no duplicates
    same_row = src[1:] == src[:-1]
    assert np.all(col[1:][same_row] > col[:-1][same_row])
    # symmetric: the multiset of (u,v) equals that of (v,u)
    fwd = np.sort(src * g.n + col)
    bwd = np.sort(col * g.n + src)
    assert np.array_equal(fwd, bwd)


@pytest.mark.parametrize("n,d,seed", [(4096, 8, 1), (1000, 4, 7), (257, 31.5, 3)])
def test_er_exact_edges(gg, n, d, seed):
    g = gg.er(n, d, seed)
    assert g.edges == int(np.floor(n * d / 2 + 0.5))
    check_simple_symmetric(g)


def test_er_deterministic_and_seed_sensitive(gg):
    a = gg.er(2000, 8, 11)
    b = gg.er(2000, 8, 11)
    c = gg.er(2000, 8, 12)
    assert np.array_equal(a.col, b.col) and np.array_equal(a.row_ptr, b.row_ptr)
    assert not np.array_equal(a.col, c.col)


def test_er_impossible(gg):
    with pytest.raises(ValueError):
        gg.er(4, 7, 1)   # 14 edges > C(4,2)


def test_grid_structure(gg):
    R, C = 5, 7
    g = gg.grid(R, C)
    assert g.n == R * C and g.edges == R * (C - 1) + (R - 1) * C
    check_simple_symmetric(g)
    for r in range(R):
        for c in range(C):
            v = r * C + c
            nb = set(g.col[g.row_ptr[v]:g.row_ptr[v + 1]].tolist())
            exp = {(r + dr) * C + (c + dc) for dr, dc in ((1, 0), (-1, 0), (0, 1), (0, -1))
                   if 0 <= r + dr < R and 0 <= c + dc < C}
            assert nb == exp


def test_rmat_structure(gg):
    g = gg.rmat(12, 16, seed=5)
    assert g.n == 4096 and 0 < g.edges <= 16 * 4096
    check_simple_symmetric(g)
    deg = g.degrees()
    # R-MAT with a=0.57 is heavily skewed: max degree far above the mean
    assert deg.max() > 10 * deg.mean()
    g2 = gg.rmat(12, 16, seed=5)
    assert np.array_equal(g.col, g2.col)


def test_weights_symmetric_and_in_range(gg):
    g = gg.add_weights(gg.er(3000, 6, 2), seed=9, lo=1, hi=1000)
    assert g.w.min() >= 1 and g.w.max() <= 1000
    src = np.repeat(np.arange(g.n), g.degrees())
    key_f = src.astype(np.int64) * g.n + g.col
    key_b = g.col.astype(np.int64) * g.n + src
    wf = dict(zip(key_f.tolist(), g.w.tolist()))
    assert all(wf[kb] == w for kb, w in zip(key_b.tolist(), g.w.tolist()))
    # roughly uniform: mean near 500.5
    assert abs(float(g.w.mean()) - 500.5) < 20


def test_uniform_bounds(gg):
    xs = [gg.uniform(5, 5, i, 3, 9) for i in range(2000)]
    assert min(xs) == 3 and max(xs) == 9
    counts = np.bincount(np.array(xs) - 3)
    assert counts.min() > 200


def test_sources_have_degree(gg):
    g = gg.disjoint_union(gg.empty(50), gg.path(10))
    s = gg.sources(g, 6, 32)
    deg = g.degrees()
    assert np.all(deg[s] >= 1)


def test_closed_form_graphs(gg):
    for g in (gg.path(6), gg.cycle(6), gg.star(6), gg.complete(6), gg.complete_bipartite(2, 3),
              gg.binary_tree(10)):
        check_simple_symmetric(g)
    assert gg.complete(6).edges == 15 and gg.cycle(6).edges == 6 and gg.binary_tree(10).edges == 9


def test_batch_sizes_recipe(gg):
    """Batched workload: instance i uses seed 1000 + i, n log-uniform in
    [2^10, 2^18), average degree uniform in [4, 32)."""
    sz = gg.batch_sizes(512, 1000)
    assert [s for _, _, s in sz] == list(range(1000, 1512))
    n = np.array([a for a, _, _ in sz])
    d = np.array([b for _, b, _ in sz])
    assert n.min() >= 1 << 10 and n.max() < 1 << 18
    assert d.min() >= 4 and d.max() < 32
    # log-uniform: half the instances below 2^14 (binomial, 5 sigma ~ 0.11)
    assert abs(np.mean(n < (1 << 14)) - 0.5) < 0.11
    assert abs(np.mean(d < 18) - 0.5) < 0.11
    assert gg.batch_sizes(3, 1000) == sz[:3]


def test_er_batch_matches_single_instances(gg):
    gs = gg.er_batch(5, 2000, workers=3, log2_hi=12.0)
    for g, (n, d, s) in zip(gs, gg.batch_sizes(5, 2000, log2_hi=12.0)):
        h = gg.er(n, d, s)
        assert g.n == n and np.array_equal(g.row_ptr, h.row_ptr) and np.array_equal(g.col, h.col)
