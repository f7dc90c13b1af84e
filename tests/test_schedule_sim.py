"""The asynchronous update rules give order-independent results under random
interleavings (CPU; the simulator is in tests/schedsim.py): BFS depths equal
the oracle's exactly, PageRank meets the one-sided bound with every residue
<= eps and its mass conserved, colourings are valid and within the rank
bound."""
import numpy as np
import pytest

import oracle
from oracle import checks
from paper_2112_00132_amd import graphgen as gg

import schedsim

D = 0.85
EPS = 1e-6


def _graphs():
    return [gg.path_graph(40), gg.star_graph(30), gg.complete_graph(12), gg.full_grid_graph(7, 9),
            gg.rmat_graph(7, 8, seed=3), gg.random_graph(150, 300, seed=6), gg.cycle_graph(25)]


GRAPHS = _graphs()


@pytest.mark.parametrize("gi", range(len(GRAPHS)), ids=[g.name for g in GRAPHS])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_bfs_any_interleaving_is_exact(gi, seed):
    g = GRAPHS[gi]
    src = gg.max_degree_vertex(g)
    np.testing.assert_array_equal(schedsim.bfs(g, src, seed), oracle.bfs(g, src))


@pytest.mark.parametrize("gi", range(len(GRAPHS)), ids=[g.name for g in GRAPHS])
@pytest.mark.parametrize("seed", [1, 2])
def test_pagerank_any_interleaving_meets_bound(gi, seed):
    g = GRAPHS[gi]
    rank, residue, _ = schedsim.pagerank(g, D, EPS, seed)
    assert residue.max(initial=0.0) <= EPS
    x, _, _, bound = oracle.pagerank(g, D)
    assert checks.pagerank_violations(g, rank, x, D, EPS, rel_tol=None, ref_bound=bound,
                                      slack_ulps=0.0) == []
    obs, exp = checks.pagerank_mass(g, rank, residue, D)
    assert abs(obs - exp) <= 1e-9 * exp


@pytest.mark.parametrize("gi", range(len(GRAPHS)), ids=[g.name for g in GRAPHS])
@pytest.mark.parametrize("order", [0, 4])
@pytest.mark.parametrize("seed", [1, 2])
def test_colouring_any_interleaving_is_valid(gi, order, seed):
    g = GRAPHS[gi]
    key = oracle.color_rank_keys(g, 3)
    col = schedsim.color(g, key, order, seed)
    assert checks.coloring_violations(g, col) == []
    assert checks.coloring_rank_violations(g, col, key) == []


@pytest.mark.parametrize("gi", range(len(GRAPHS)), ids=[g.name for g in GRAPHS])
def test_colouring_all_ordered_is_unique(gi):
    """With every vertex of degree >= 1 ordered, any interleaving gives
    first-fit in rank order, the oracle's colouring."""
    g = GRAPHS[gi]
    key = oracle.color_rank_keys(g, 5)
    ref, _, _ = oracle.color_fifo(g, 5, order_degree=1)
    for seed in (1, 2):
        np.testing.assert_array_equal(schedsim.color(g, key, 1, seed), ref)


def test_simulator_interleaves_heavily():
    """The simulator really scrambles the order: different seeds start
    different numbers of PageRank tasks."""
    g = GRAPHS[5]
    counts = {schedsim.pagerank(g, D, EPS, s)[2] for s in (1, 2, 3, 4)}
    assert len(counts) > 1
