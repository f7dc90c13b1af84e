"""Parity at the workloads' full sizes, in the launch configurations the
benchmark times (a ring per XCD; workgroup workers of 1024 threads taking
256 tasks, 512 for BFS on R-MAT; colouring with 512-thread workers; PageRank
on R-MAT persistent with residue combining, and also in rounds inside one
launch without it and as discrete launches).

- R-MAT scale 22 (permuted, int32 CSR): BFS depths equal the oracle's
  exactly; PageRank (with residue combining, and without it in rounds)
  meets the stated bound against the FP64 oracle with every residue <= eps
  and mass conserved; the colouring is proper, within the rank bound and
  within 10% of sequential greedy's colour count.
- 2048^2 road-like grid: BFS exact, PageRank within the bound.
- 640 batched instances: every BFS instance exact, a sample of PageRank
  instances within the bound.
"""
import numpy as np
import pytest

import oracle
from oracle import checks
from paper_2112_00132_amd import graphgen as gg

pytestmark = pytest.mark.gpu

D = 0.85
EPS = 1e-7
CFG = dict(worker=1024, fetch=256, timeout_ms=60000)
# the benchmark's BFS on R-MAT, and colouring with the library's default rule
CFG_BFS_RMAT = dict(worker=1024, fetch=512, timeout_ms=60000)
CFG_GC_RMAT = dict(worker=512, fetch=256, timeout_ms=60000)
# the benchmark's colouring rule on R-MAT: every neighbour's colour avoided, the
# ~sqrt(n) highest-degree vertices coloured in rank order, fixed claims
CFG_GC_RMAT_SQRT = dict(worker=512, fetch=256, fetch_policy=1, color_forbid_all=1,
                        color_order_degree=-2, timeout_ms=60000)
# the benchmark's PageRank on R-MAT: persistent, shallowest-ring pushes, claims of
# up to 128 tasks, lists over 2,048 edges split on the hub board, residue
# combining (the default)
CFG_PR_RMAT = dict(worker=1024, fetch=128, split_degree=2048, push_policy=2, timeout_ms=60000)
# without combining, in rounds inside one persistent launch
CFG_PR_RMAT_PLAIN = dict(strategy=3, worker=1024, fetch=256, split_degree=2048, push_policy=1,
                         pr_combine=-1, timeout_ms=60000)
# the same as discrete launches, the last few-task rounds as one persistent launch
CFG_PR_RMAT_DISCRETE = dict(strategy=2, worker=1024, fetch=256, discrete_tail=65536, timeout_ms=60000)


def _atos():
    import paper_2112_00132_amd as atos
    return atos


@pytest.fixture(scope="module")
def rmat22():
    g = gg.rmat_graph(22, 16, seed=1, permute_seed=2)
    return g, gg.max_degree_vertex(g)


@pytest.fixture(scope="module")
def grid2048():
    g = gg.grid_graph(2048, seed=1)
    return g, gg.random_source(g, 1)


_PR_REF = {}


def _pr_check(g, rank, res):
    if g.name not in _PR_REF:  # the FP64 fixed point, once per graph
        _PR_REF[g.name] = oracle.pagerank(g, D, threads=16)
    x, _, _, bound = _PR_REF[g.name]
    r = rank.cpu().numpy().astype(np.float64)
    rr = res.cpu().numpy().astype(np.float64)
    assert rr.max(initial=0.0) <= float(np.float32(EPS))
    v = checks.pagerank_violations(g, r, x, D, EPS, ref_bound=bound)
    assert v == [], v
    obs, exp = checks.pagerank_mass(g, r, rr, D)
    assert abs(obs - exp) <= 1e-5 * exp


def test_rmat22_bfs_pagerank_color(rmat22):
    import torch
    atos = _atos()
    g, src = rmat22
    dg = atos.Graph.from_csr(g.offsets, g.cols, offsets_int64=False)
    depth = atos.bfs(dg, src, cfg=atos.Config(**CFG_BFS_RMAT))
    np.testing.assert_array_equal(depth.cpu().numpy(), oracle.bfs(g, src))
    res = torch.empty(g.n, dtype=torch.float32, device="cuda")
    rank, st = atos.pagerank(dg, D, EPS, cfg=atos.Config(**CFG_PR_RMAT), residual=res, stats=True)
    _pr_check(g, rank, res)
    assert 0 < st.combine_atomics < st.combined_updates < st.edges_scanned
    col, ncol = atos.color(dg, 3, cfg=atos.Config(**CFG_GC_RMAT))
    c = col.cpu().numpy()
    assert checks.coloring_violations(g, c) == []
    assert checks.coloring_rank_violations(g, c, oracle.color_rank_keys(g, 3)) == []
    _, kseq = oracle.greedy_color(g)
    assert int(ncol.item()) == c.max() + 1
    assert c.max() + 1 <= 1.1 * kseq, (c.max() + 1, kseq)


def test_rmat22_color_sqrt_class(rmat22):
    """The benchmark's colouring rule: every neighbour's colour avoided and an
    ordered class of the ~sqrt(n) highest-degree vertices; proper, colours <=
    degree, within 10% of sequential greedy."""
    atos = _atos()
    g, _ = rmat22
    dg = atos.Graph.from_csr(g.offsets, g.cols, offsets_int64=False)
    col, ncol = atos.color(dg, 3, cfg=atos.Config(**CFG_GC_RMAT_SQRT))
    c = col.cpu().numpy()
    assert checks.coloring_violations(g, c) == []
    assert (c <= np.diff(g.offsets)).all()
    _, kseq = oracle.greedy_color(g)
    assert int(ncol.item()) == c.max() + 1
    assert c.max() + 1 <= 1.1 * kseq, (c.max() + 1, kseq)


def test_rmat22_pagerank_uncombined_rounds(rmat22):
    """Every edge update a device atomic, in rounds inside one launch."""
    import torch
    atos = _atos()
    g, _ = rmat22
    dg = atos.Graph.from_csr(g.offsets, g.cols, offsets_int64=False)
    res = torch.empty(g.n, dtype=torch.float32, device="cuda")
    rank, st = atos.pagerank(dg, D, EPS, cfg=atos.Config(**CFG_PR_RMAT_PLAIN), residual=res,
                             stats=True)
    _pr_check(g, rank, res)
    assert st.combined_updates == 0 and st.rounds > 1


def test_rmat22_pagerank_discrete(rmat22):
    """Discrete launches with the last few-task rounds as one persistent
    launch: within the bound like every other strategy."""
    import torch
    atos = _atos()
    g, _ = rmat22
    dg = atos.Graph.from_csr(g.offsets, g.cols, offsets_int64=False)
    res = torch.empty(g.n, dtype=torch.float32, device="cuda")
    rank, st = atos.pagerank(dg, D, EPS, cfg=atos.Config(**CFG_PR_RMAT_DISCRETE), residual=res,
                             stats=True)
    _pr_check(g, rank, res)
    assert st.rounds > 1


def test_grid2048_bfs_pagerank(grid2048):
    import torch
    atos = _atos()
    g, src = grid2048
    dg = atos.Graph.from_csr(g.offsets, g.cols, offsets_int64=False)
    cfg = atos.Config(**CFG)
    depth = atos.bfs(dg, src, cfg=cfg)
    np.testing.assert_array_equal(depth.cpu().numpy(), oracle.bfs(g, src))
    res = torch.empty(g.n, dtype=torch.float32, device="cuda")
    # the benchmark's PageRank on the grid: shallowest-ring pushes, 512-task claims
    rank = atos.pagerank(dg, D, EPS, cfg=atos.Config(worker=1024, fetch=512, push_policy=2,
                                                     timeout_ms=60000), residual=res)
    _pr_check(g, rank, res)


def test_batch640_instances():
    import types
    import torch
    atos = _atos()
    w = gg.batch_workload(n_graphs=640, n_pagerank=128, seed=4, device="cuda")
    dg = atos.Graph(w.offsets, w.cols)
    b = atos.Batch(dg, w.instances, D, EPS, cfg=atos.Config(**CFG))
    res = torch.zeros(w.n, dtype=torch.float32, device="cuda")
    state, st = b.run(residual=res, stats=True)
    assert st.status == 0
    state_h = state.cpu()
    res_h = res.cpu().numpy().astype(np.float64)
    pr_checked = 0
    rng = np.random.default_rng(7)
    pr_sample = set(rng.choice([k for k, i in enumerate(w.instances) if i[0] == 2], 8,
                               replace=False).tolist())
    for k, (app, vb, ve, _src) in enumerate(w.instances):
        o, c, lsrc = w.local[k]
        if app == 2 and k not in pr_sample:
            continue
        oh = o.cpu().numpy().astype(np.int64)
        hg = types.SimpleNamespace(n=oh.size - 1, offsets=oh, cols=c.cpu().numpy().astype(np.int32))
        if app == 1:
            np.testing.assert_array_equal(state_h[vb:ve].numpy(), oracle.bfs(hg, lsrc),
                                          err_msg=f"instance {k} {w.kinds[k]}")
        else:
            rank = state_h[vb:ve].view(torch.float32).numpy().astype(np.float64)
            x, _, _, bound = oracle.pagerank(hg, D, threads=16)
            assert res_h[vb:ve].max(initial=0.0) <= float(np.float32(EPS))
            v = checks.pagerank_violations(hg, rank, x, D, EPS, ref_bound=bound)
            assert v == [], (k, w.kinds[k], v)
            pr_checked += 1
    assert pr_checked == len(pr_sample)
    b.close()
