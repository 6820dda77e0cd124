"""The all-core CPU baselines (OpenMP level-synchronous BFS and frontier
Bellman-Ford) give the oracle's answer on every graph family the benchmark
and the tests use, at several thread counts. They are timed beside the
oracle by the benchmark, so they must be exact, not only fast."""
import numpy as np
import pytest

import oracle


def graphs(gg):
    yield gg.er(3000, 8, 1)
    yield gg.rmat(14, 16, seed=3)
    yield gg.grid(64, 50)
    yield gg.path(500)
    yield gg.disjoint_union(gg.er(300, 4, 2), gg.empty(7))
    yield gg.star(200)


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_bfs_parallel_equals_oracle(gg, threads):
    for g in graphs(gg):
        for src in (0, g.n // 2, g.n - 1):
            got, used = oracle.bfs_parallel(g, src, threads)
            assert used == threads
            assert np.array_equal(got, oracle.bfs(g, src)), (g.name, src)


@pytest.mark.parametrize("threads", [1, 4, 8])
def test_sssp_parallel_equals_oracle(gg, threads):
    for g in graphs(gg):
        gw = gg.add_weights(g, 7, 1, 1000)
        for src in (0, g.n - 1):
            got, used = oracle.sssp_parallel(gw, src, threads)
            assert used == threads
            assert np.array_equal(got, oracle.sssp(gw, src)), (g.name, src)


def test_parallel_rejects_bad_source(gg):
    g = gg.er(100, 4, 1)
    with pytest.raises(oracle.OracleError):
        oracle.bfs_parallel(g, 100)
