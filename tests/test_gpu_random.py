"""Randomised GPU parity (hypothesis): random small graphs, sources and launch
shapes (worker size, FETCH, ring layout, publishing ring, strategy); BFS
bit-exact, PageRank within its bound, colourings valid and rank-bounded."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings, strategies as st

import oracle
from oracle import checks
from paper_2112_00132_amd import graphgen as gg

pytestmark = pytest.mark.gpu

D = 0.85
EPS = 1e-7


def _atos():
    import paper_2112_00132_amd as atos
    return atos


graphs = st.one_of(
    st.builds(lambda n, m, s: gg.random_graph(n, m, seed=s), st.integers(1, 300), st.integers(0, 900),
              st.integers(0, 1 << 30)),
    st.builds(lambda sc, ef, s: gg.rmat_graph(sc, ef, seed=s), st.integers(4, 9), st.integers(1, 16),
              st.integers(0, 1 << 30)),
    st.builds(lambda a, b: gg.full_grid_graph(a, b), st.integers(1, 20), st.integers(1, 20)),
)
shapes = st.tuples(st.sampled_from([64, 128, 256, 512, 1024]), st.integers(1, 256),
                   st.sampled_from([0, 1, 2]), st.sampled_from([0, 1, 2]), st.sampled_from([0, 2]))


@settings(max_examples=40, deadline=None, suppress_health_check=list(HealthCheck))
@given(g=graphs, shape=shapes, pick=st.integers(0, 1 << 30))
def test_random_graphs_and_shapes(g, shape, pick):
    import torch
    atos = _atos()
    worker, fetch, layout, push, strategy = shape
    fetch = min(fetch, worker)
    cfg = atos.Config(strategy=strategy, worker=worker, fetch=fetch, queue_layout=layout,
                      push_policy=push, timeout_ms=20000)
    dg = atos.Graph.from_csr(g.offsets, g.cols, offsets_int64=bool(pick & 1))
    src = pick % g.n
    np.testing.assert_array_equal(atos.bfs(dg, src, cfg=cfg).cpu().numpy(), oracle.bfs(g, src))
    res = torch.empty(g.n, dtype=torch.float32, device="cuda")
    rank = atos.pagerank(dg, D, EPS, cfg=cfg, residual=res)
    assert res.max().item() <= float(np.float32(EPS))
    x, _, _, bound = oracle.pagerank(g, D)
    assert checks.pagerank_violations(g, rank.cpu().numpy().astype(np.float64), x, D, EPS,
                                      ref_bound=bound) == []
    col, ncol = atos.color(dg, seed=pick & 0xFFFF, cfg=cfg)
    c = col.cpu().numpy()
    assert checks.coloring_violations(g, c) == []
    assert checks.coloring_rank_violations(g, c, oracle.color_rank_keys(g, pick & 0xFFFF)) == []
    assert int(ncol.item()) == (c.max() + 1 if g.n else 0)
