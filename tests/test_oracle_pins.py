"""Pins for the CPU oracle: each oracle routine is checked against something
other than itself -- brute force on every tiny graph, closed forms, library
routines (scipy, numpy.linalg, networkx) and hand-worked fixtures -- chosen
so that a dropped term, a wrong sign or index or a transposed operand in the
oracle fails at least one of them."""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
from oracle import checks
from paper_2112_00132_amd import graphgen as gg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
D = 0.85


def _graph_from_edges(n, edges):
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    return gg.csr_from_edges(n, e[:, 0], e[:, 1])


def _dense_adj(g):
    a = np.zeros((g.n, g.n))
    src, dst = g.edge_list()
    a[src, dst] = 1.0
    return a


def _floyd_warshall_hops(g):
    n = g.n
    inf = 10 ** 9
    dist = np.full((n, n), inf, dtype=np.int64)
    np.fill_diagonal(dist, 0)
    src, dst = g.edge_list()
    dist[src, dst] = np.minimum(dist[src, dst], 1)
    for k in range(n):
        dist = np.minimum(dist, dist[:, [k]] + dist[[k], :])
    dist[dist >= inf] = -1
    return dist


def _solve_pagerank(g, damping, teleport):
    a = _dense_adj(g)
    deg = a.sum(axis=0)
    m = a / np.where(deg > 0, deg, 1.0)[None, :]  # column-normalised A D^-1
    return np.linalg.solve(np.eye(g.n) - damping * m, (1 - damping) * teleport)


# ----------------------------------------------------------------- BFS
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_bfs_brute_force_all_graphs(n):
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        edges = [p for i, p in enumerate(pairs) if mask >> i & 1]
        g = _graph_from_edges(n, edges) if edges else gg.empty_graph(n)
        fw = _floyd_warshall_hops(g)
        for s in range(n):
            np.testing.assert_array_equal(oracle.bfs(g, s), fw[s], err_msg=f"edges={edges} s={s}")


def test_bfs_brute_force_random_6_to_9():
    rng = np.random.default_rng(11)
    for trial in range(400):
        n = int(rng.integers(6, 10))
        g = gg.random_graph(n, int(rng.integers(0, 2 * n)), seed=trial)
        fw = _floyd_warshall_hops(g)
        s = int(rng.integers(0, n))
        np.testing.assert_array_equal(oracle.bfs(g, s), fw[s])


@pytest.mark.parametrize("make", [lambda: gg.rmat_graph(10, 8, seed=3),
                                  lambda: gg.rmat_graph(12, 16, seed=4, permute_seed=2),
                                  lambda: gg.grid_graph(64, seed=5),
                                  lambda: gg.random_graph(3000, 4000, seed=6)])
def test_bfs_vs_scipy(make):
    import scipy.sparse as sp
    from scipy.sparse.csgraph import shortest_path
    g = make()
    mat = sp.csr_matrix((np.ones(g.m), g.cols, g.offsets), shape=(g.n, g.n))
    for s in [gg.max_degree_vertex(g), 0, g.n - 1]:
        ref = shortest_path(mat, method="D", unweighted=True, indices=s)
        ref = np.where(np.isinf(ref), -1, ref).astype(np.int32)
        got = oracle.bfs(g, s)
        np.testing.assert_array_equal(got, ref)
        assert checks.bfs_certificate(g, s, got) == []


def test_bfs_closed_forms():
    rows, cols = 13, 17
    g = gg.full_grid_graph(rows, cols)
    for s in [0, 5 * cols + 7, rows * cols - 1]:
        si, sj = divmod(s, cols)
        ii, jj = np.divmod(np.arange(rows * cols), cols)
        np.testing.assert_array_equal(oracle.bfs(g, s), np.abs(ii - si) + np.abs(jj - sj))
    g = gg.path_graph(50)
    np.testing.assert_array_equal(oracle.bfs(g, 20), np.abs(np.arange(50) - 20))
    g = gg.star_graph(9)
    np.testing.assert_array_equal(oracle.bfs(g, 0), [0] + [1] * 9)
    np.testing.assert_array_equal(oracle.bfs(g, 4), [1, 2, 2, 2, 0, 2, 2, 2, 2, 2])
    g = gg.complete_graph(7)
    np.testing.assert_array_equal(oracle.bfs(g, 3), [1, 1, 1, 0, 1, 1, 1])
    g = gg.empty_graph(5)
    np.testing.assert_array_equal(oracle.bfs(g, 2), [-1, -1, 0, -1, -1])


@pytest.mark.parametrize("make", [lambda: gg.rmat_graph(12, 16, seed=4, permute_seed=2),
                                  lambda: gg.grid_graph(96, seed=5),
                                  lambda: gg.path_graph(500),
                                  lambda: gg.random_graph(3000, 4000, seed=6)])
def test_bfs_levelsync_equals_scipy(make):
    """The OpenMP level-synchronous BFS (CPU timing leg) against scipy, at
    several thread counts."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import shortest_path
    g = make()
    mat = sp.csr_matrix((np.ones(g.m), g.cols, g.offsets), shape=(g.n, g.n))
    for s in [gg.max_degree_vertex(g), g.n - 1]:
        ref = shortest_path(mat, method="D", unweighted=True, indices=s)
        ref = np.where(np.isinf(ref), -1, ref).astype(np.int32)
        for threads in (1, 4):
            np.testing.assert_array_equal(oracle.bfs_levelsync(g, s, threads), ref)


def test_bfs_rejects_bad_source():
    with pytest.raises(ValueError):
        oracle.bfs(gg.path_graph(4), 4)
    with pytest.raises(ValueError):
        oracle.bfs(gg.path_graph(4), -1)


def test_bfs_certificate_rejects_mutations():
    g = gg.grid_graph(32, seed=2)
    s = 17
    d = oracle.bfs(g, s)
    assert checks.bfs_certificate(g, s, d) == []
    far = int(np.argmax(d))
    for mutate in (lambda x: x.__setitem__(far, x[far] + 1),
                   lambda x: x.__setitem__(far, x[far] - 1),
                   lambda x: x.__setitem__(s, 1),
                   lambda x: x.__setitem__(far, -1),
                   lambda x: x.__setitem__(slice(None), x + 1)):
        bad = d.copy()
        mutate(bad)
        assert checks.bfs_certificate(g, s, bad) != []


# ----------------------------------------------------------------- PageRank
def test_pagerank_vs_linear_solve_tiny():
    rng = np.random.default_rng(5)
    for trial in range(60):
        n = int(rng.integers(1, 25))
        g = gg.random_graph(n, int(rng.integers(0, 3 * n)), seed=100 + trial)
        x, it, delta, bound = oracle.pagerank(g, D, tol=1e-13)
        ref = _solve_pagerank(g, D, np.ones(g.n))
        assert delta < 1e-13
        np.testing.assert_allclose(x, ref, rtol=0, atol=1e-10)
        assert (np.abs(x - ref) <= bound + 1e-13).all()


@pytest.mark.parametrize("g", [gg.cycle_graph(11), gg.torus_graph(6, 9), gg.complete_graph(8)])
def test_pagerank_regular_graph_is_all_ones(g):
    x, *_ = oracle.pagerank(g, D)
    np.testing.assert_allclose(x, 1.0, rtol=0, atol=1e-12)


@pytest.mark.parametrize("k", [1, 3, 10, 1000])
def test_pagerank_star_closed_form(k):
    x, *_ = oracle.pagerank(gg.star_graph(k), D)
    leaf = (1 + D / k) / (1 + D)
    centre = (1 - D) + D * (k + D) / (1 + D)
    np.testing.assert_allclose(x[0], centre, rtol=1e-12)
    np.testing.assert_allclose(x[1:], leaf, rtol=1e-12)


def test_pagerank_isolated_vertices_keep_teleport():
    g = _graph_from_edges(6, [[0, 1], [1, 2]])  # 3, 4, 5 isolated
    x, *_ = oracle.pagerank(g, D)
    np.testing.assert_allclose(x[3:], 1 - D, rtol=0, atol=1e-15)


def test_pagerank_vs_networkx():
    import networkx as nx
    for seed in range(4):
        g = gg.largest_component(gg.rmat_graph(9, 8, seed=seed + 1))
        G = nx.Graph()
        G.add_nodes_from(range(g.n))
        G.add_edges_from(zip(*(a.tolist() for a in g.edge_list())))
        pr = nx.pagerank(G, alpha=D, tol=1e-15, max_iter=10000)
        ref = np.array([pr[v] for v in range(g.n)]) * g.n
        x, *_ = oracle.pagerank(g, D)
        np.testing.assert_allclose(x, ref, rtol=1e-8)


def test_pagerank_mass_identity():
    g = gg.rmat_graph(12, 8, seed=7)
    x, *_ = oracle.pagerank(g, D)
    obs, exp = checks.pagerank_mass(g, x, None, D)
    assert abs(obs - exp) <= 1e-9 * exp


def test_ppr_mass_identity():
    """Personalized mass closed form: 1 for a source with neighbours, 1-d for an
    isolated one (its x is (1-d) e_s)."""
    g = gg.rmat_graph(11, 8, seed=5)
    deg = np.diff(g.offsets)
    for s in (int(np.argmax(deg)), int(np.flatnonzero(deg == 1)[0]), int(np.flatnonzero(deg == 0)[0])):
        x, *_ = oracle.ppr(g, s, D)
        obs, exp = checks.ppr_mass(g, s, x, np.zeros(g.n), D)
        assert exp == (1.0 if deg[s] > 0 else 1.0 - D)
        assert abs(obs - exp) <= 1e-9


def test_pagerank_thread_count_does_not_change_result():
    g = gg.rmat_graph(12, 16, seed=8)
    a, ia, *_ = oracle.pagerank(g, D, threads=1)
    b, ib, *_ = oracle.pagerank(g, D, threads=4)
    assert ia == ib
    np.testing.assert_array_equal(a, b)


def test_personalized_pagerank_vs_solve_and_networkx():
    import networkx as nx
    rng = np.random.default_rng(9)
    for trial in range(20):
        n = int(rng.integers(2, 30))
        g = gg.random_graph(n, int(rng.integers(1, 3 * n)), seed=300 + trial)
        s = int(gg.max_degree_vertex(g))
        e = np.zeros(g.n)
        e[s] = 1.0
        x, *_ = oracle.ppr(g, s, D)
        np.testing.assert_allclose(x, _solve_pagerank(g, D, e), rtol=0, atol=1e-12)
    g = gg.largest_component(gg.rmat_graph(8, 8, seed=3))
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    G.add_edges_from(zip(*(a.tolist() for a in g.edge_list())))
    s = 5
    pr = nx.pagerank(G, alpha=D, personalization={s: 1.0}, tol=1e-15, max_iter=10000)
    x, *_ = oracle.ppr(g, s, D)
    np.testing.assert_allclose(x, [pr[v] for v in range(g.n)], rtol=1e-7, atol=1e-14)


def test_push_bsp_oracle_bounds_and_mass():
    """The sequential bulk-synchronous push (the paper's Algorithm 3 order)
    ends with every residue <= eps, its rank obeys the one-sided truncation
    bound against the fixed point, and rank + residue/(1-d) conserves mass."""
    for g in (gg.rmat_graph(12, 8, seed=1), gg.grid_graph(48, seed=3), gg.star_graph(50)):
        eps = 1e-7
        rank, res, rounds, pushes, pops = oracle.pagerank_push_bsp(g, D, eps)
        x, _, _, bound = oracle.pagerank(g, D)
        assert rounds > 0 and pushes > 0 and pops >= g.n
        assert res.max() <= eps
        obs, exp = checks.pagerank_mass(g, rank, res, D)
        assert abs(obs - exp) <= 1e-9 * exp
        assert checks.pagerank_violations(g, rank, x, D, eps, ref_bound=bound) == []


def test_pagerank_checker_rejects_mutations():
    g = gg.grid_graph(40, seed=4)
    x, _, _, bound = oracle.pagerank(g, D)
    rank, *_ = oracle.pagerank_push_bsp(g, D, 1e-7)
    assert checks.pagerank_violations(g, rank, x, D, 1e-7, ref_bound=bound) == []
    for delta in (+2e-5, -2e-5):
        bad = rank.copy()
        bad[7] += delta
        assert checks.pagerank_violations(g, bad, x, D, 1e-7, ref_bound=bound) != []
    i = int(np.argmin(x))  # x(i) < 1, so the tolerance there is an absolute 1e-5
    bad = rank.copy()
    bad[i] = x[i] + 9e-6  # within the tolerance but above the fixed point beyond FP32 slack
    assert checks.pagerank_violations(g, bad, x, D, 1e-7, ref_bound=bound) != []


# ----------------------------------------------------------------- colouring
def test_greedy_matches_networkx_id_order():
    import networkx as nx
    for g in (gg.rmat_graph(10, 8, seed=2), gg.grid_graph(30, seed=1),
              gg.random_graph(500, 2000, seed=3), gg.rmat_graph(11, 16, seed=5, permute_seed=2)):
        G = nx.Graph()
        G.add_nodes_from(range(g.n))
        G.add_edges_from(zip(*(a.tolist() for a in g.edge_list())))
        ref = nx.greedy_color(G, strategy=lambda G_, colors: sorted(G_.nodes()))
        color, k = oracle.greedy_color(g)
        np.testing.assert_array_equal(color, [ref[v] for v in range(g.n)])
        assert k == color.max() + 1
        assert checks.coloring_violations(g, color) == []


def test_greedy_closed_forms():
    assert oracle.greedy_color(gg.complete_graph(9))[1] == 9
    assert oracle.greedy_color(gg.cycle_graph(9))[1] == 3
    assert oracle.greedy_color(gg.cycle_graph(10))[1] == 2
    assert oracle.greedy_color(gg.star_graph(12))[1] == 2
    assert oracle.greedy_color(gg.path_graph(7))[1] == 2
    rows, cols = 9, 14
    color, k = oracle.greedy_color(gg.full_grid_graph(rows, cols))
    ii, jj = np.divmod(np.arange(rows * cols), cols)
    assert k == 2
    np.testing.assert_array_equal(color, (ii + jj) % 2)
    color, k = oracle.greedy_color(gg.empty_graph(4))
    assert k == 1 and (color == 0).all()


def test_coloring_checker_rejects_mutations():
    g = gg.rmat_graph(10, 8, seed=2)
    color, _ = oracle.greedy_color(g)
    assert checks.coloring_violations(g, color) == []
    u = int(gg.max_degree_vertex(g))
    w = int(g.cols[g.offsets[u]])
    bad = color.copy()
    bad[u] = bad[w]
    assert checks.coloring_violations(g, bad) != []
    bad = color.copy()
    bad[3] = -1
    assert checks.coloring_violations(g, bad) != []


# ----------------------------------------------------------------- hand-worked fixtures
@pytest.mark.parametrize("name", ["petersen.json", "star3.json"])
def test_golden_fixtures(name):
    with open(os.path.join(GOLDEN, name)) as f:
        fx = json.load(f)
    n = 1 + max(max(e) for e in fx["edges"])
    g = _graph_from_edges(n, fx["edges"])
    np.testing.assert_array_equal(oracle.bfs(g, fx["bfs_source"]), fx["bfs_depth"])
    color, k = oracle.greedy_color(g)
    np.testing.assert_array_equal(color, fx["greedy_color"])
    assert k == fx["greedy_ncolors"]
    x, *_ = oracle.pagerank(g, fx["pagerank_damping"])
    np.testing.assert_allclose(x, fx["pagerank"], rtol=1e-12)


# ----------------------------------------------------------------- speculative colouring (FIFO)
@pytest.mark.parametrize("make", [lambda: gg.rmat_graph(12, 8, seed=1, permute_seed=2),
                                  lambda: gg.grid_graph(40, seed=2),
                                  lambda: gg.random_graph(800, 3000, seed=5),
                                  lambda: gg.full_grid_graph(9, 13)])
def test_color_fifo_valid_and_rank_bounded(make):
    g = make()
    color, k, tasks = oracle.color_fifo(g, 3)
    key = oracle.color_rank_keys(g, 3)
    assert checks.coloring_violations(g, color) == []
    assert checks.coloring_rank_violations(g, color, key) == []
    assert k == color.max() + 1
    assert tasks >= 2 * g.n  # every vertex is assigned and checked at least once
    top = int(np.lexsort((np.arange(g.n), key))[-1])
    assert color[top] == 0  # the top-ranked vertex never yields


def test_color_fifo_complete_graph_is_rank_order():
    """On K_n every vertex sees every other: the colour of v is the number of
    vertices that outrank it, whatever the schedule."""
    g = gg.complete_graph(37)
    color, k, _ = oracle.color_fifo(g, 11)
    key = oracle.color_rank_keys(g, 11).astype(np.int64)
    order = np.lexsort((np.arange(g.n), key))[::-1]  # highest rank first
    expect = np.empty(g.n, dtype=np.int64)
    expect[order] = np.arange(g.n)
    np.testing.assert_array_equal(color, expect)
    assert k == 37


def test_color_fifo_star_and_rank_keys():
    g = gg.star_graph(25)
    color, k, _ = oracle.color_fifo(g, 3)
    assert color[0] == 0 and (color[1:] == 1).all() and k == 2  # the hub outranks its leaves
    key = oracle.color_rank_keys(g, 3)
    assert (key[0] >> 16) == 25 and ((key[1:] >> 16) == 1).all()  # degree in the high half
    assert len(set((key & 0xFFFF).tolist())) > 20  # pseudo-random low half


def _first_fit_in_rank_order(g, key, members):
    """Textbook greedy colouring of the subgraph induced by `members`, taking
    vertices from the highest rank (key, id) down."""
    order = [int(v) for v in np.lexsort((np.arange(g.n), key.astype(np.int64)))[::-1] if members[v]]
    color = np.full(g.n, -1, dtype=np.int64)
    for v in order:
        used = {int(color[w]) for w in g.cols[g.offsets[v]:g.offsets[v + 1]] if members[w] and w != v}
        c = 0
        while c in used:
            c += 1
        color[v] = c
    return color


@pytest.mark.parametrize("make", [lambda: gg.rmat_graph(11, 8, seed=1, permute_seed=2),
                                  lambda: gg.grid_graph(30, seed=2),
                                  lambda: gg.random_graph(500, 2500, seed=5)])
def test_color_fifo_ordered_class_is_greedy_in_rank_order(make):
    """With every vertex of degree >= 1 in the ordered class, each is coloured
    once, after all its outranking neighbours: first-fit in rank order.  Task
    count: n initial assigns, one wake-up per vertex that had to wait, and a
    check task only for the isolated vertices (a class vertex checks inside
    its assign task)."""
    g = make()
    key = oracle.color_rank_keys(g, 3)
    color, k, tasks = oracle.color_fifo(g, 3, order_degree=1)
    deg = np.diff(g.offsets)
    ref = _first_fit_in_rank_order(g, key, deg >= 1)
    np.testing.assert_array_equal(color[deg >= 1], ref[deg >= 1])
    assert (color[deg == 0] == 0).all()
    src = np.repeat(np.arange(g.n), deg)
    k64 = key.astype(np.int64)
    up = (k64[g.cols] > k64[src]) | ((k64[g.cols] == k64[src]) & (g.cols > src))
    waited = np.bincount(src[up & (g.cols != src)], minlength=g.n) > 0
    assert tasks == g.n + int(waited.sum()) + int((deg == 0).sum())


def test_color_fifo_mixed_classes():
    """Degree >= 8 ordered, the rest speculative: valid and rank-bounded, and
    the ordered class alone is first-fit in rank order on its induced subgraph
    (its outranking neighbours are all in the class)."""
    g = gg.rmat_graph(12, 8, seed=1, permute_seed=2)
    key = oracle.color_rank_keys(g, 3)
    color, k, tasks = oracle.color_fifo(g, 3, order_degree=8)
    assert checks.coloring_violations(g, color) == []
    assert checks.coloring_rank_violations(g, color, key) == []
    cls = np.minimum(np.diff(g.offsets), 0xFFFF) >= 8
    ref = _first_fit_in_rank_order(g, key, cls)
    np.testing.assert_array_equal(color[cls], ref[cls])
    _, _, tasks_spec = oracle.color_fifo(g, 3)
    assert tasks < tasks_spec  # the ordered class never recolours


def test_rank_checker_rejects_id_order_greedy():
    """ID-order greedy ignores ranks, so it breaks the rank bound somewhere."""
    g = gg.rmat_graph(12, 8, seed=1, permute_seed=2)
    color, _ = oracle.greedy_color(g)
    assert checks.coloring_rank_violations(g, color, oracle.color_rank_keys(g, 3)) != []


# ----------------------------------------------------------------- push-BSP work counts
def test_push_bsp_first_round_counts():
    """Round 1 pops every vertex once (the first frontier is all of V) and
    pushes along every stored edge once: pops = n, edge pushes = sum of
    degrees, on any graph (isolated vertices pop and push nothing)."""
    for g in (gg.rmat_graph(11, 8, seed=3), gg.grid_graph(40, seed=2), gg.star_graph(17),
              gg.empty_graph(6), gg.random_graph(300, 700, seed=9)):
        _, _, rounds, pushes, pops = oracle.pagerank_push_bsp(g, D, 1e-7, max_rounds=1)
        assert rounds == 1
        assert pops == g.n
        assert pushes == int(np.diff(g.offsets).sum())


@pytest.mark.parametrize("eps", [1e-3, 1e-5, 1e-7, 3e-9])
def test_push_bsp_single_edge_closed_form(eps):
    """Two vertices joined by one edge (a cycle of length 2).  Both start with
    residue (1-d) d.  Round 1: vertex 0 pops and gives d(1-d)d to vertex 1,
    which then pops (1-d)d(1+d) and gives d times that back; from then on one
    vertex pops per round and the residue shrinks by d each time, so after
    round j the only residue is (1-d) d^(j+1) (1+d).  The run stops after the
    first round R with (1-d) d^(R+1) (1+d) <= eps, with R + 1 pops and R + 1
    edge pushes."""
    import math
    g = gg.path_graph(2)
    c = (1 - D) * D * (1 + D)
    r_real = math.log(eps / c) / math.log(D)  # (1-d) d^(R+1)(1+d) = eps at R + 1 = this + 1
    assert abs(r_real - round(r_real)) > 1e-6  # eps is not at a rounding boundary
    R = max(1, math.ceil(r_real))
    rank, res, rounds, pushes, pops = oracle.pagerank_push_bsp(g, D, eps)
    assert rounds == R
    assert pops == R + 1 and pushes == R + 1
    assert res.max() <= eps


def test_push_bsp_star_hand_worked():
    """Hand-worked run on a 4-leaf star with damping 0.5 (every value dyadic,
    so exact in FP64); derivation in the fixture."""
    with open(os.path.join(GOLDEN, "star4_push_bsp.json")) as f:
        fx = json.load(f)
    g = _graph_from_edges(5, fx["edges"])
    for case in fx["cases"]:
        rank, res, rounds, pushes, pops = oracle.pagerank_push_bsp(g, fx["damping"], case["epsilon"])
        assert (rounds, pops, pushes) == (case["rounds"], case["pops"], case["edge_pushes"])
        np.testing.assert_array_equal(rank, case["rank"])
        np.testing.assert_array_equal(res, case["residue"])


# ----------------------------------------------------------------- FIFO colouring, hand trace
def _fmix64_priority(seed, v):
    """MurmurHash3's 64-bit finaliser of seed ^ (golden-ratio constant * (v+1)), low 32 bits."""
    m = (1 << 64) - 1
    k = seed ^ ((0x9E3779B97F4A7C15 * (v + 1)) & m)
    k ^= k >> 33
    k = (k * 0xFF51AFD7ED558CCD) & m
    k ^= k >> 33
    k = (k * 0xC4CEB9FE1A85EC53) & m
    k ^= k >> 33
    return k & 0xFFFFFFFF


def test_color_rank_keys_match_published_hash():
    g = gg.rmat_graph(10, 8, seed=2, permute_seed=2)
    key = oracle.color_rank_keys(g, 12345)
    deg = np.diff(g.offsets)
    for v in range(0, g.n, 7):
        assert int(key[v]) == (min(int(deg[v]), 0xFFFF) << 16) | (_fmix64_priority(12345, v) >> 16)


def test_color_fifo_hand_traced():
    """Algorithm 6 by one FIFO worker on a 6-vertex graph, traced by hand
    (tests/golden/color_fifo6.json): colours, colour count and the 18 tasks
    (6 assigns, 6 checks, 2 recolours after lost conflicts, their 2 checks,
    one recolour of a lower-ranked neighbour and its check)."""
    with open(os.path.join(GOLDEN, "color_fifo6.json")) as f:
        fx = json.load(f)
    g = _graph_from_edges(6, fx["edges"])
    deg = np.diff(g.offsets)
    keys = [(min(int(deg[v]), 0xFFFF) << 16) | (_fmix64_priority(fx["seed"], v) >> 16) for v in range(6)]
    assert sorted(range(6), key=lambda v: (keys[v], v), reverse=True) == fx["rank_order_high_to_low"]
    color, k, tasks = oracle.color_fifo(g, fx["seed"], order_degree=0)
    np.testing.assert_array_equal(color, fx["colors"])
    assert k == fx["ncolors"]
    assert tasks == fx["tasks"]
