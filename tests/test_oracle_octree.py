"""Pins of the octree oracle (the work-stealing workload), against a
verifier that characterises the result without building a tree: the leaves
are exactly the cubes that hold at most `cap` points (or are at depth 21)
and whose parent cube holds more; they tile the output in order of their
codes, and inside a leaf the points keep their input order. Together these
fix the output uniquely, so any correct builder must produce it."""
import numpy as np
import pytest

import oracle

BITS = 21


def morton(x, y, z):
    """63-bit codes: per level (most significant first) the child index
    4 bx + 2 by + bz."""
    x = x.astype(np.uint64)
    y = y.astype(np.uint64)
    z = z.astype(np.uint64)
    code = np.zeros(len(x), dtype=np.uint64)
    for b in range(BITS - 1, -1, -1):
        child = (((x >> np.uint64(b)) & np.uint64(1)) << np.uint64(2)) | \
                (((y >> np.uint64(b)) & np.uint64(1)) << np.uint64(1)) | ((z >> np.uint64(b)) & np.uint64(1))
        code = (code << np.uint64(3)) | child
    return code


def check_octree(x, y, z, cap, out, leaves):
    n = len(x)
    assert out.shape == (n, 4) and out.dtype == np.uint32
    idx = out[:, 3].astype(np.int64)
    assert np.array_equal(np.sort(idx), np.arange(n)), "not a permutation"
    assert np.array_equal(out[:, 0], x[idx]) and np.array_equal(out[:, 1], y[idx]) and \
        np.array_equal(out[:, 2], z[idx]), "coordinates do not travel with their index"
    if n == 0:
        assert len(leaves) == 0
        return
    first, end, depth = leaves[:, 0].astype(np.int64), leaves[:, 1].astype(np.int64), leaves[:, 2].astype(np.int64)
    code = leaves[:, 3].astype(np.uint64) | (leaves[:, 4].astype(np.uint64) << np.uint64(32))
    assert first[0] == 0 and end[-1] == n and np.all(end > first), "leaves must tile [0, n) without gaps"
    assert np.array_equal(first[1:], end[:-1])
    assert np.all(depth <= BITS)
    full = morton(out[:, 0], out[:, 1], out[:, 2])
    all_codes = np.sort(morton(x, y, z))
    shift = (3 * (BITS - depth)).astype(np.uint64)
    for k in range(len(leaves)):
        seg = full[first[k]:end[k]] >> shift[k]
        assert np.all(seg == code[k]), f"leaf {k} holds a point outside its cube"
        size = end[k] - first[k]
        assert size <= cap or depth[k] == BITS, f"leaf {k} is too large"
        assert np.all(np.diff(idx[first[k]:end[k]]) > 0), f"leaf {k} does not keep the input order"
        if depth[k] > 0:
            # the parent cube must hold more than cap points (else it would be the leaf)
            ps = shift[k] + np.uint64(3)
            lo = (code[k] >> np.uint64(3)) << ps
            hi = lo + (np.uint64(1) << ps)
            inside = np.searchsorted(all_codes, hi, "left") - np.searchsorted(all_codes, lo, "left")
            assert inside > cap, f"leaf {k}'s parent holds only {inside} points"
    # cubes in code order (a leaf's extended prefix strictly increases)
    ext = code << shift
    assert np.all(np.diff(ext.astype(np.float64)) >= 0) and np.all(ext[1:] > ext[:-1])


@pytest.mark.parametrize("kind,n,cap,seed", [("uniform", 5000, 8, 1), ("uniform", 20000, 32, 2),
                                             ("clustered", 20000, 16, 3), ("clustered", 3000, 1, 4)])
def test_octree_characterisation(gg, kind, n, cap, seed):
    x, y, z = gg.points(n, seed, kind)
    out, leaves = oracle.octree(x, y, z, cap)
    check_octree(x, y, z, cap, out, leaves)


def test_octree_closed_forms():
    # at most cap points: one leaf, the root
    x = np.array([5, 1, 9], dtype=np.uint32)
    out, leaves = oracle.octree(x, x, x, 3)
    assert leaves.tolist() == [[0, 3, 0, 0, 0]] and out[:, 3].tolist() == [0, 1, 2]
    # identical points never separate: one leaf at the deepest level
    p = np.full(10, 12345, dtype=np.uint32)
    out, leaves = oracle.octree(p, p, p, 2)
    assert leaves.shape == (1, 5) and leaves[0, :3].tolist() == [0, 10, 21]
    assert out[:, 3].tolist() == list(range(10))
    # the 8 corners of the cube, one point per child at depth 1, listed in
    # child-index order whatever the input order
    s = (1 << 21) - 1
    corners = [(s, 0, s), (0, 0, 0), (s, s, s), (0, s, 0), (0, 0, s), (s, 0, 0), (0, s, s), (s, s, 0)]
    cx, cy, cz = (np.array(c, dtype=np.uint32) for c in zip(*corners))
    out, leaves = oracle.octree(cx, cy, cz, 1)
    assert leaves[:, 2].tolist() == [1] * 8 and leaves[:, 3].tolist() == list(range(8))
    child = [4 * (a > 0) + 2 * (b > 0) + (c > 0) for a, b, c in corners]
    assert out[:, 3].tolist() == list(np.argsort(child))
    # empty input
    e = np.zeros(0, dtype=np.uint32)
    out, leaves = oracle.octree(e, e, e, 4)
    assert out.shape == (0, 4) and leaves.shape[0] == 0


def test_octree_brute_force_small(gg):
    """A plain recursive build on a few hundred points, written from the
    definition with Python lists (no stable-sort shortcuts), agrees."""
    x, y, z = gg.points(300, 7, "clustered")
    cap = 3
    pts = [(int(x[i]), int(y[i]), int(z[i]), i) for i in range(300)]
    order, leaves = [], []

    def build(p, depth, code):
        if len(p) <= cap or depth == BITS:
            if p:
                leaves.append((len(order), len(order) + len(p), depth, code))
                order.extend(p)
            return
        b = BITS - 1 - depth
        for c in range(8):
            sub = [q for q in p if (((q[0] >> b) & 1) << 2 | ((q[1] >> b) & 1) << 1 | ((q[2] >> b) & 1)) == c]
            build(sub, depth + 1, code * 8 + c)

    build(pts, 0, 0)
    out, lv = oracle.octree(x, y, z, cap)
    assert [tuple(r) for r in out.tolist()] == order
    assert [(a, b, d, lo | (hi << 32)) for a, b, d, lo, hi in lv.tolist()] == leaves


def test_octree_verifier_catches_planted_errors(gg):
    x, y, z = gg.points(4000, 5, "uniform")
    out, leaves = oracle.octree(x, y, z, 8)
    check_octree(x, y, z, 8, out, leaves)
    # two points of one leaf swapped: order inside the leaf broken
    k = int(np.argmax(leaves[:, 1] - leaves[:, 0]))
    bad = out.copy()
    f = int(leaves[k, 0])
    bad[[f, f + 1]] = bad[[f + 1, f]]
    with pytest.raises(AssertionError):
        check_octree(x, y, z, 8, bad, leaves)
    # a leaf split in two (its parent would then be a valid leaf): minimality
    if leaves[k, 1] - leaves[k, 0] >= 2:
        f, e, d, lo, hi = (int(v) for v in leaves[k])
        code = lo | (hi << 32)
        pts = out[f:e]
        codes = morton(pts[:, 0], pts[:, 1], pts[:, 2]) >> np.uint64(3 * (BITS - d - 1))
        if len(set(codes.tolist())) > 1:
            split = int(np.argmax(codes != codes[0]))
            rows = [[f, f + split, d + 1, int(codes[0]) & 0xFFFFFFFF, int(codes[0]) >> 32],
                    [f + split, e, d + 1, int(codes[split]) & 0xFFFFFFFF, int(codes[split]) >> 32]]
            bad_leaves = np.concatenate([leaves[:k], np.array(rows, dtype=np.uint32), leaves[k + 1:]])
            with pytest.raises(AssertionError):
                check_octree(x, y, z, 8, out, bad_leaves)
    # wrong cube code on a leaf
    bad_leaves = leaves.copy()
    bad_leaves[0, 3] ^= 1
    with pytest.raises(AssertionError):
        check_octree(x, y, z, 8, out, bad_leaves)
