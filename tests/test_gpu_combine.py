"""GPU parity of PageRank with residue combining (atos_config.pr_combine).

The residue updates of the highest-degree vertices are summed in a table in
each worker's LDS and reach the device residue with one atomic per vertex and
flush, whose old value takes the threshold-crossing decision on the sum (with
Algorithm 4's rule a flush only adds the sums and the sweeps enqueue).  The
fixed point, the one-sided truncation bound and the mass identity are those
of the plain run (only the order of FP64 additions differs), so every case
here is held to the same checks as the plain PageRank parity tests, and the
counters must account for the combined updates."""
import numpy as np
import pytest

import oracle
from oracle import checks
from paper_2112_00132_amd import graphgen as gg

pytestmark = pytest.mark.gpu

D = 0.85
EPS = 1e-7
TABLE = 12288  # slots of a worker's table
MIN_DEGREE = 64  # lowest degree a combined vertex can have


def _atos():
    import paper_2112_00132_amd as atos
    return atos


def _circulant(n, half):
    """Every vertex joined to the `half` next and previous ones: degree 2*half."""
    i = np.repeat(np.arange(n, dtype=np.int64), half)
    k = np.tile(np.arange(1, half + 1, dtype=np.int64), n)
    return gg.csr_from_edges(n, i, (i + k) % n, f"circ{n}x{2 * half}")


def _double_star(leaves):
    n = 2 + 2 * leaves
    src = [0] + [0] * leaves + [1] * leaves
    dst = [1] + list(range(2, 2 + leaves)) + list(range(2 + leaves, n))
    return gg.csr_from_edges(n, np.array(src), np.array(dst), f"dstar{leaves}")


def _graphs():
    return [
        gg.star_graph(700),
        _double_star(3000),
        gg.rmat_graph(12, 16, seed=4, permute_seed=2),
        gg.rmat_graph(14, 16, seed=5),
        gg.grid_graph(64, seed=5),  # no vertex of degree >= 64: an empty table
    ]


GRAPHS = _graphs()


def _check(g, rank, res):
    x, _, _, bound = oracle.pagerank(g, D)
    r = rank.cpu().numpy().astype(np.float64)
    rr = res.cpu().numpy().astype(np.float64)
    assert rr.max(initial=0.0) <= float(np.float32(EPS)), f"residue {rr.max()} > eps"
    v = checks.pagerank_violations(g, r, x, D, EPS, ref_bound=bound)
    assert v == [], v
    obs, exp = checks.pagerank_mass(g, r, rr, D)
    assert abs(obs - exp) <= 1e-5 * exp


def _combinable(g):
    return bool((np.diff(g.offsets) >= MIN_DEGREE).any())


def _counters_consistent(g, st):
    if _combinable(g):
        assert 0 < st.combine_atomics <= st.combined_updates <= st.edges_scanned
    else:
        assert st.combined_updates == 0 and st.combine_atomics == 0


@pytest.mark.parametrize("gi", range(len(GRAPHS)), ids=[g.name for g in GRAPHS])
@pytest.mark.parametrize("strategy", ["persistent", "rounds", "discrete", "check_size"])
@pytest.mark.parametrize("window", [1, 300, 131072])
def test_combined_pagerank_within_bound(gi, strategy, window):
    """Every strategy that runs the worker kernel, and Algorithm 4's sweep
    rule (Check_Size 4), with flush windows from one edge (a flush after every
    batch) to the default."""
    import torch
    atos = _atos()
    g = GRAPHS[gi]
    dg = atos.Graph.from_csr(g.offsets, g.cols, offsets_int64=(gi % 2 == 1))
    s = {"persistent": atos.PERSISTENT, "rounds": atos.ROUNDS, "discrete": atos.DISCRETE,
         "check_size": atos.PERSISTENT}[strategy]
    cfg = atos.Config(strategy=s, worker=1024, fetch=256, pr_combine=window, timeout_ms=20000,
                      pr_check_size=4 if strategy == "check_size" else 0)
    res = torch.empty(g.n, dtype=torch.float32, device="cuda")
    rank, st = atos.pagerank(dg, D, EPS, cfg=cfg, residual=res, stats=True)
    _check(g, rank, res)
    _counters_consistent(g, st)


@pytest.mark.parametrize("worker,fetch", [(64, 16), (256, 64), (512, 256)])
def test_combined_pagerank_smaller_workers(worker, fetch):
    """Combining asked for explicitly on the smaller worker sizes (one
    workgroup per CU, as the table fills the LDS)."""
    import torch
    atos = _atos()
    for g in (GRAPHS[1], GRAPHS[2]):
        dg = atos.Graph.from_csr(g.offsets, g.cols)
        cfg = atos.Config(worker=worker, fetch=fetch, pr_combine=4096, split_degree=300,
                          timeout_ms=20000)
        res = torch.empty(g.n, dtype=torch.float32, device="cuda")
        rank, st = atos.pagerank(dg, D, EPS, cfg=cfg, residual=res, stats=True)
        _check(g, rank, res)
        _counters_consistent(g, st)
        assert st.hub_posts > 0  # chunks of the board combine too


def test_default_is_on_for_1024_thread_workers_only():
    import torch
    atos = _atos()
    g = GRAPHS[2]
    dg = atos.Graph.from_csr(g.offsets, g.cols)
    res = torch.empty(g.n, dtype=torch.float32, device="cuda")
    for worker, on in ((1024, True), (512, False)):
        rank, st = atos.pagerank(dg, D, EPS, cfg=atos.Config(worker=worker), residual=res, stats=True)
        _check(g, rank, res)
        assert (st.combined_updates > 0) == on
    rank, st = atos.pagerank(dg, D, EPS, cfg=atos.Config(worker=1024, pr_combine=-1), residual=res,
                             stats=True)
    _check(g, rank, res)
    assert st.combined_updates == 0 and st.combine_atomics == 0


def test_table_filled_from_a_class_larger_than_it():
    """A 64-regular graph of 20,000 vertices: every vertex is in the lowest
    degree class, which holds more vertices than the table has slots, so the
    table is filled from that class (12,288 of the 20,000 vertices).  About
    that share of all updates is combined: none would be if whole classes
    only were taken, all would be if the slots were overrun."""
    import torch
    atos = _atos()
    g = _circulant(20000, 32)
    assert set(np.diff(g.offsets).tolist()) == {64}
    dg = atos.Graph.from_csr(g.offsets, g.cols)
    res = torch.empty(g.n, dtype=torch.float32, device="cuda")
    rank, st = atos.pagerank(dg, D, EPS, cfg=atos.Config(worker=1024, pr_combine=131072),
                             residual=res, stats=True)
    _check(g, rank, res)
    share = st.combined_updates / st.edges_scanned
    assert abs(share - TABLE / g.n) < 0.08, share


def test_combining_refused_where_it_cannot_run():
    atos = _atos()
    g = GRAPHS[0]
    dg = atos.Graph.from_csr(g.offsets, g.cols)
    with pytest.raises(atos.AtosError) as err:
        atos.pagerank(dg, D, EPS, cfg=atos.Config(pr_combine=4096, strategy=atos.BSP))
    assert err.value.status == 8
    with pytest.raises(atos.AtosError) as err:
        atos.ppr(dg, 3, D, EPS, cfg=atos.Config(pr_combine=4096))
    assert err.value.status == 8
    for call in (lambda: atos.bfs(dg, 0, cfg=atos.Config(pr_combine=4096)),
                 lambda: atos.color(dg, 3, cfg=atos.Config(pr_combine=4096))):
        with pytest.raises(atos.AtosError) as err:
            call()
        assert err.value.status == 8
    with pytest.raises(atos.AtosError) as err:
        atos.pagerank(dg, D, EPS, cfg=atos.Config(pr_combine=-2))
    assert err.value.status == 1
    # the defaults stay valid where combining does not apply
    atos.ppr(dg, 3, D, EPS)
    atos.pagerank(dg, D, EPS, cfg=atos.Config(strategy=atos.BSP))


def test_combined_then_plain_calls_share_a_workspace():
    """Calls with and without combining alternate on one graph (and so on one
    cached workspace): each meets the bound."""
    import torch
    atos = _atos()
    g = GRAPHS[3]
    dg = atos.Graph.from_csr(g.offsets, g.cols)
    res = torch.empty(g.n, dtype=torch.float32, device="cuda")
    for comb in (131072, -1, 1, 0, -1):
        rank = atos.pagerank(dg, D, EPS, cfg=atos.Config(worker=1024, pr_combine=comb), residual=res)
        _check(g, rank, res)
