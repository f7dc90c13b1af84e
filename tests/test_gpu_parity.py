"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

BFS depths must be bit-exact.  PageRank must lie within 1e-5*max(1, x) of the
FP64 fixed point and obey the one-sided truncation bound; every final
residue must be <= eps.  Colourings must be proper, use colours <= degree,
and (on graphs large enough for the bound to mean something) at most 10%
more colours than sequential greedy."""
import numpy as np
import pytest

import oracle
from oracle import checks
from paper_2112_00132_amd import graphgen as gg

pytestmark = pytest.mark.gpu

D = 0.85
EPS = 1e-7


def _atos():
    import paper_2112_00132_amd as atos
    return atos


def _dev(g, int64=True):
    atos = _atos()
    return atos.Graph.from_csr(g.offsets, g.cols, offsets_int64=int64)


def _small_graphs():
    return [
        gg.path_graph(200),
        gg.star_graph(700),
        gg.complete_graph(24),
        gg.full_grid_graph(30, 41),
        gg.rmat_graph(10, 8, seed=3),
        gg.rmat_graph(12, 16, seed=4, permute_seed=2),
        gg.grid_graph(64, seed=5),
        gg.random_graph(5000, 6000, seed=6),
    ]


SMALL = _small_graphs()
WORKER_FETCH = [(64, 1), (64, 64), (256, 7), (256, 64), (1024, 256)]


def _sources(g):
    return sorted({gg.max_degree_vertex(g), 0, g.n - 1})


# ------------------------------------------------------------------ BFS
@pytest.mark.parametrize("gi", range(len(SMALL)), ids=[g.name for g in SMALL])
@pytest.mark.parametrize("worker,fetch", WORKER_FETCH)
def test_bfs_persistent_small(gi, worker, fetch):
    atos = _atos()
    g = SMALL[gi]
    dg = _dev(g, int64=(gi % 2 == 0))
    cfg = atos.Config(worker=worker, fetch=fetch, timeout_ms=20000)
    for s in _sources(g):
        depth, st = atos.bfs(dg, s, cfg=cfg, stats=True)
        ref = oracle.bfs(g, s)
        np.testing.assert_array_equal(depth.cpu().numpy(), ref, err_msg=f"{g.name} s={s}")
        assert st.tasks_popped >= int((ref >= 0).sum())


@pytest.mark.parametrize("gi", range(len(SMALL)), ids=[g.name for g in SMALL])
@pytest.mark.parametrize("worker", [64, 256])
def test_bfs_bsp_small(gi, worker):
    atos = _atos()
    g = SMALL[gi]
    dg = _dev(g)
    cfg = atos.Config(strategy=atos.BSP, worker=worker)
    for s in _sources(g):
        depth, st = atos.bfs(dg, s, cfg=cfg, stats=True)
        ref = oracle.bfs(g, s)
        np.testing.assert_array_equal(depth.cpu().numpy(), ref)
        assert st.rounds == ref.max() + 1  # one round per level, the last one empty-handed
        assert st.tasks_popped == int((ref >= 0).sum())  # level-synchronous: no overwork


def test_bfs_degenerate_graphs():
    atos = _atos()
    for g, s in ((gg.empty_graph(1), 0), (gg.empty_graph(50), 17), (gg.path_graph(2), 1)):
        dg = _dev(g)
        for strategy in (atos.PERSISTENT, atos.BSP, atos.DISCRETE, atos.ROUNDS):
            depth = atos.bfs(dg, s, cfg=atos.Config(strategy=strategy))
            np.testing.assert_array_equal(depth.cpu().numpy(), oracle.bfs(g, s))


def test_bfs_rejects_bad_source():
    atos = _atos()
    dg = _dev(gg.path_graph(5))
    for bad in (-1, 5):
        with pytest.raises(atos.AtosError) as e:
            atos.bfs(dg, bad)
        assert e.value.status == 1


def test_bfs_repeated_calls_reuse_workspace():
    """Ring positions continue across calls on one workspace; results stay exact."""
    atos = _atos()
    g = gg.rmat_graph(12, 8, seed=9)
    dg = _dev(g)
    cfg = atos.Config(worker=256, fetch=32)
    srcs = [gg.max_degree_vertex(g), 5, 100, 4000, gg.max_degree_vertex(g)]
    for s in srcs * 3:
        np.testing.assert_array_equal(atos.bfs(dg, s, cfg=cfg).cpu().numpy(), oracle.bfs(g, s))


def test_bfs_config0_rmat16():
    """R-MAT scale 16, edge factor 8, source = highest-degree vertex."""
    atos = _atos()
    g = gg.rmat_graph(16, 8, seed=1)
    assert g.n == 65536
    s = gg.max_degree_vertex(g)
    ref = oracle.bfs(g, s)
    for int64 in (True, False):
        dg = _dev(g, int64=int64)
        for cfg in (atos.Config(), atos.Config(worker=64, fetch=16),
                    atos.Config(strategy=atos.BSP)):
            depth = atos.bfs(dg, s, cfg=cfg).cpu().numpy()
            np.testing.assert_array_equal(depth, ref)
            assert checks.bfs_certificate(g, s, depth) == []


def test_overflow_is_reported_and_next_run_recovers():
    """A single worker cannot drain a 1024-slot ring while it pushes 5000 tasks."""
    atos = _atos()
    g = gg.star_graph(5000)
    dg = _dev(g)
    cfg = atos.Config(grid=1, worker=64, queue_capacity=1024, timeout_ms=20000)
    for stats in (True, False):  # raised with or without the counters
        with pytest.raises(atos.AtosError) as e:
            atos.bfs(dg, 0, cfg=cfg, stats=stats, overflow_retries=0)
        assert e.value.status == 3
    assert dg.last_status(atos.APP_BFS, cfg).status == 3
    np.testing.assert_array_equal(atos.bfs(dg, 0).cpu().numpy(), oracle.bfs(g, 0))


def test_overflow_retried_with_larger_rings():
    """The binding reruns an overflowed call with twice the ring capacity:
    1024 -> 2048 -> 4096 -> 8192 slots, the last one large enough."""
    atos = _atos()
    g = gg.star_graph(5000)
    dg = _dev(g)
    cfg = atos.Config(grid=1, worker=64, queue_capacity=1024, timeout_ms=20000)
    depth = atos.bfs(dg, 0, cfg=cfg, overflow_retries=3)
    np.testing.assert_array_equal(depth.cpu().numpy(), oracle.bfs(g, 0))


def test_host_abort_stops_the_run_and_next_run_recovers():
    """A host thread sets the abort flag while a long run is on the GPU: the
    workers (or the level-synchronous loop) stop, the call reports EABORTED,
    and the next call on the same workspace is exact."""
    import threading
    atos = _atos()
    g = gg.full_grid_graph(2, 200000)  # 200k dependent levels: seconds of work
    dg = _dev(g)
    flag = atos.AbortFlag()
    try:
        for strategy in (atos.PERSISTENT, atos.BSP):
            flag.clear()
            cfg = atos.Config(strategy=strategy, abort=flag, timeout_ms=30000)
            timer = threading.Timer(0.2, flag.set)
            timer.start()
            with pytest.raises(atos.AtosError) as e:
                atos.bfs(dg, 0, cfg=cfg, stats=True)
            timer.join()
            assert e.value.status == 5, strategy
            flag.clear()
            h = gg.path_graph(300)
            np.testing.assert_array_equal(atos.bfs(_dev(h), 0, cfg=cfg).cpu().numpy(),
                                          oracle.bfs(h, 0))
            np.testing.assert_array_equal(
                atos.bfs(dg, 7, cfg=atos.Config(strategy=strategy, abort=flag)).cpu().numpy()[:10],
                oracle.bfs(g, 7)[:10])
    finally:
        flag.close()


def test_timeout_is_reported_and_next_run_recovers():
    atos = _atos()
    g = gg.full_grid_graph(2, 200000)  # 200k levels: far more than 1 ms of work
    dg = _dev(g)
    cfg = atos.Config(timeout_ms=1)
    with pytest.raises(atos.AtosError) as e:
        atos.bfs(dg, 0, cfg=cfg, stats=True)
    assert e.value.status == 4
    h = gg.path_graph(300)
    dh = _dev(h)
    np.testing.assert_array_equal(atos.bfs(dh, 0).cpu().numpy(), oracle.bfs(h, 0))


# ------------------------------------------------------------------ PageRank
def _check_pr(g, rank, residual):
    x, _, _, bound = oracle.pagerank(g, D)
    r = rank.cpu().numpy().astype(np.float64)
    res = residual.cpu().numpy().astype(np.float64)
    assert res.max(initial=0.0) <= float(np.float32(EPS)), f"residue {res.max()} > eps"
    v = checks.pagerank_violations(g, r, x, D, EPS, ref_bound=bound)
    assert v == [], v
    obs, exp = checks.pagerank_mass(g, r, res, D)
    assert abs(obs - exp) <= 1e-5 * exp


@pytest.mark.parametrize("gi", range(len(SMALL)), ids=[g.name for g in SMALL])
@pytest.mark.parametrize("worker,fetch", [(64, 16), (256, 64), (1024, 128)])
def test_pagerank_persistent_small(gi, worker, fetch):
    import torch
    atos = _atos()
    g = SMALL[gi]
    dg = _dev(g, int64=(gi % 2 == 1))
    res = torch.empty(g.n, dtype=torch.float32, device="cuda")
    rank = atos.pagerank(dg, D, EPS, cfg=atos.Config(worker=worker, fetch=fetch, timeout_ms=20000),
                         residual=res)
    _check_pr(g, rank, res)


@pytest.mark.parametrize("gi", range(len(SMALL)), ids=[g.name for g in SMALL])
def test_pagerank_bsp_small(gi):
    import torch
    atos = _atos()
    g = SMALL[gi]
    dg = _dev(g)
    res = torch.empty(g.n, dtype=torch.float32, device="cuda")
    rank = atos.pagerank(dg, D, EPS, cfg=atos.Config(strategy=atos.BSP), residual=res)
    _check_pr(g, rank, res)


@pytest.mark.parametrize("gi", range(len(SMALL)), ids=[g.name for g in SMALL])
@pytest.mark.parametrize("check_size,worker,fetch", [(1, 64, 16), (4, 256, 64), (16, 1024, 256)])
def test_pagerank_sweep_small(gi, check_size, worker, fetch):
    """Algorithm 4's enqueue rule (pr_check_size > 0): edge updates push no
    task, sweeps of Check_Size positions per task do, and the run ends after
    a clean sweep of every vertex; same bound as the threshold-crossing rule."""
    import torch
    atos = _atos()
    g = SMALL[gi]
    dg = _dev(g, int64=(gi % 2 == 0))
    res = torch.empty(g.n, dtype=torch.float32, device="cuda")
    cfg = atos.Config(worker=worker, fetch=fetch, pr_check_size=check_size, timeout_ms=20000)
    rank, st = atos.pagerank(dg, D, EPS, cfg=cfg, residual=res, stats=True)
    _check_pr(g, rank, res)
    assert st.rounds >= 1  # launches: the last one's clean sweep found nothing
    assert st.tasks_popped >= g.n  # every vertex starts queued


def test_segmented_layout_is_for_batches_only():
    atos = _atos()
    dg = _dev(gg.path_graph(50))
    cfg = atos.Config(queue_layout=atos.QUEUE_SEGMENTED)
    for call in (lambda: atos.bfs(dg, 0, cfg=cfg), lambda: atos.pagerank(dg, D, EPS, cfg=cfg),
                 lambda: atos.color(dg, 3, cfg=cfg)):
        with pytest.raises(atos.AtosError) as err:
            call()
        assert err.value.status == 8


def test_pagerank_sweep_refused_where_unsupported():
    atos = _atos()
    dg = _dev(gg.path_graph(50))
    for cfg in (atos.Config(pr_check_size=4, strategy=atos.BSP),
                atos.Config(pr_check_size=4, strategy=atos.DISCRETE)):
        with pytest.raises(atos.AtosError) as err:
            atos.pagerank(dg, D, EPS, cfg=cfg)
        assert err.value.status == 8
    with pytest.raises(atos.AtosError) as err:
        atos.ppr(dg, 3, D, EPS, cfg=atos.Config(pr_check_size=4))
    assert err.value.status == 8
    with pytest.raises(atos.AtosError) as err:
        atos.pagerank(dg, D, EPS, cfg=atos.Config(pr_check_size=-1))
    assert err.value.status == 1


def test_pagerank_degenerate_and_closed_forms():
    import torch
    atos = _atos()
    for g in (gg.empty_graph(7), gg.cycle_graph(100), gg.star_graph(3), gg.torus_graph(20, 30)):
        dg = _dev(g)
        for strategy in (atos.PERSISTENT, atos.BSP, atos.DISCRETE, atos.ROUNDS):
            res = torch.empty(g.n, dtype=torch.float32, device="cuda")
            rank = atos.pagerank(dg, D, EPS, cfg=atos.Config(strategy=strategy), residual=res)
            _check_pr(g, rank, res)


def test_pagerank_rejects_bad_arguments():
    atos = _atos()
    dg = _dev(gg.path_graph(5))
    for d, e in ((0.0, 1e-7), (1.0, 1e-7), (0.85, 0.0), (0.85, -1.0)):
        with pytest.raises(atos.AtosError) as err:
            atos.pagerank(dg, d, e)
        assert err.value.status == 1
    g = gg.path_graph(5)
    import torch
    directed = atos.Graph(torch.as_tensor(g.offsets).cuda(), torch.as_tensor(g.cols).cuda(),
                          symmetric=False)
    with pytest.raises(atos.AtosError) as err:
        atos.pagerank(directed)
    assert err.value.status == 7


# ------------------------------------------------------------------ colouring
def _check_gc(g, col, ncol, tight, seed=3):
    c = col.cpu().numpy()
    assert checks.coloring_violations(g, c) == []
    assert checks.coloring_rank_violations(g, c, oracle.color_rank_keys(g, seed)) == []
    k = int(ncol.cpu().numpy()[0])
    assert k == int(c.max(initial=-1)) + 1
    _, kseq = oracle.greedy_color(g)
    if tight:
        assert k <= int(np.floor(1.10 * kseq)), (k, kseq)
    return k


@pytest.mark.parametrize("gi", range(len(SMALL)), ids=[g.name for g in SMALL])
@pytest.mark.parametrize("worker,fetch", [(64, 1), (64, 32), (256, 64)])
def test_color_persistent_small(gi, worker, fetch):
    atos = _atos()
    g = SMALL[gi]
    dg = _dev(g)
    col, ncol = atos.color(dg, seed=3, cfg=atos.Config(worker=worker, fetch=fetch, timeout_ms=20000))
    _check_gc(g, col, ncol, tight=False)


@pytest.mark.parametrize("gi", range(len(SMALL)), ids=[g.name for g in SMALL])
@pytest.mark.parametrize("strategy,worker,fetch", [(0, 64, 1), (0, 256, 64), (0, 1024, 256),
                                                   (1, 256, 0)])
@pytest.mark.parametrize("order", [0, -2, 8])
def test_color_forbid_all_small(gi, strategy, worker, fetch, order):
    """Assignments that avoid every neighbour's colour (Algorithms 5/6 as
    printed), with no ordered class, with the ~sqrt(n) highest-degree vertices
    as the class, and with every vertex of degree >= 8: a proper colouring
    with colours <= degree; the rank bound of the default rule does not
    apply."""
    atos = _atos()
    g = SMALL[gi]
    dg = _dev(g)
    cfg = atos.Config(strategy=strategy, worker=worker, fetch=fetch, color_forbid_all=1,
                      color_order_degree=order, timeout_ms=20000)
    col, ncol = atos.color(dg, seed=3, cfg=cfg)
    c = col.cpu().numpy()
    assert checks.coloring_violations(g, c) == []
    assert int(ncol.cpu().numpy()[0]) == int(c.max(initial=-1)) + 1
    assert (c <= np.diff(g.offsets)).all()


def test_color_sqrt_class_within_band_rmat16():
    """Every neighbour's colour avoided with the ~sqrt(n) class on R-MAT scale
    16: proper, colours <= degree, and within 10% of sequential first-fit
    (persistent and level-synchronous)."""
    atos = _atos()
    g = gg.rmat_graph(16, 8, seed=1)
    dg = _dev(g, int64=False)
    _, kseq = oracle.greedy_color(g)
    for strategy, worker in ((atos.PERSISTENT, 0), (atos.BSP, 256)):
        cfg = atos.Config(strategy=strategy, worker=worker, color_forbid_all=1, color_order_degree=-2,
                          timeout_ms=20000)
        col, ncol = atos.color(dg, seed=3, cfg=cfg)
        c = col.cpu().numpy()
        assert checks.coloring_violations(g, c) == []
        assert (c <= np.diff(g.offsets)).all()
        assert c.max() + 1 <= 1.1 * kseq, (strategy, c.max() + 1, kseq)
    with pytest.raises(atos.AtosError) as err:
        atos.color(dg, seed=3, cfg=atos.Config(color_order_degree=-3))
    assert err.value.status == 1


@pytest.mark.parametrize("gi", range(len(SMALL)), ids=[g.name for g in SMALL])
def test_color_bsp_small(gi):
    atos = _atos()
    g = SMALL[gi]
    dg = _dev(g)
    col, ncol = atos.color(dg, seed=3, cfg=atos.Config(strategy=atos.BSP))
    _check_gc(g, col, ncol, tight=False)


def test_color_config0_bound():
    atos = _atos()
    g = gg.rmat_graph(16, 8, seed=1, permute_seed=2)
    dg = _dev(g)
    for cfg in (atos.Config(), atos.Config(worker=256, fetch=64), atos.Config(strategy=atos.BSP)):
        col, ncol = atos.color(dg, seed=3, cfg=cfg)
        _check_gc(g, col, ncol, tight=True)


def test_color_degenerate():
    atos = _atos()
    for g in (gg.empty_graph(5), gg.complete_graph(40), gg.cycle_graph(9)):
        dg = _dev(g)
        for strategy in (atos.PERSISTENT, atos.BSP, atos.DISCRETE, atos.ROUNDS):
            col, ncol = atos.color(dg, cfg=atos.Config(strategy=strategy))
            k = _check_gc(g, col, ncol, tight=False)
            if g.name.startswith("complete"):
                assert k == 40


@pytest.mark.parametrize("order", [-1, 8, 32])
@pytest.mark.parametrize("gi", [2, 4, 5, 6, 7], ids=[SMALL[i].name for i in (2, 4, 5, 6, 7)])
def test_color_single_sequential_worker_equals_fifo_oracle(gi, order):
    """One wavefront worker taking one task at a time is the FIFO schedule of
    the speculative colouring: colours and task count match the oracle, with
    and without the ordered class."""
    atos = _atos()
    g = SMALL[gi]
    # one shared ring: with a ring per XCD the single worker's pops would not be FIFO
    cfg = atos.Config(worker=64, fetch=1, grid=1, queue_layout=atos.QUEUE_GLOBAL,
                      color_order_degree=order)
    col, ncol, st = atos.color(_dev(g), seed=3, cfg=cfg, stats=True)
    ref, k, tasks = oracle.color_fifo(g, 3, order_degree=max(order, 0))
    np.testing.assert_array_equal(col.cpu().numpy(), ref)
    assert int(ncol.item()) == k
    assert st.tasks_popped == tasks


@pytest.mark.parametrize("strategy", [0, 1, 2])
@pytest.mark.parametrize("gi", range(len(SMALL)), ids=[g.name for g in SMALL])
def test_color_all_ordered_is_first_fit_in_rank_order(gi, strategy):
    """With every vertex of degree >= 1 in the ordered class the colouring is
    unique whatever the schedule (first-fit in rank order), so the concurrent
    run must equal the oracle exactly."""
    atos = _atos()
    g = SMALL[gi]
    cfg = atos.Config(strategy=strategy, color_order_degree=1, timeout_ms=20000)
    col, ncol = atos.color(_dev(g, int64=(gi % 2 == 0)), seed=5, cfg=cfg)
    ref, k, _ = oracle.color_fifo(g, 5, order_degree=1)
    np.testing.assert_array_equal(col.cpu().numpy(), ref)
    assert int(ncol.item()) == (k if g.n else 0)


@pytest.mark.parametrize("strategy", [0, 1, 2])
def test_color_complete_graph_is_rank_order_under_concurrency(strategy):
    """On K_n the outcome does not depend on the schedule: colour = number of
    outranking vertices.  Pins the rank keys under full concurrency."""
    atos = _atos()
    g = gg.complete_graph(200)
    col, ncol = atos.color(_dev(g), seed=11, cfg=atos.Config(strategy=strategy))
    ref, _, _ = oracle.color_fifo(g, 11)
    np.testing.assert_array_equal(col.cpu().numpy(), ref)
    assert int(ncol.item()) == 200


@pytest.mark.parametrize("gi", [1, 2, 4, 5, 7], ids=[SMALL[i].name for i in (1, 2, 4, 5, 7)])
def test_color_hub_board_single_worker_equals_fifo_oracle(gi):
    """A threshold of 8 edges sends most colouring tasks through the hub board
    (chunks whose colour masks are ORed, finish run by the completing chunk);
    one worker taking one task at a time still follows the FIFO schedule
    exactly."""
    atos = _atos()
    g = SMALL[gi]
    cfg = atos.Config(worker=64, fetch=1, grid=1, queue_layout=atos.QUEUE_GLOBAL, split_degree=8,
                      color_order_degree=32)
    col, ncol, st = atos.color(_dev(g), seed=3, cfg=cfg, stats=True)
    ref, k, tasks = oracle.color_fifo(g, 3, order_degree=32)
    np.testing.assert_array_equal(col.cpu().numpy(), ref)
    assert int(ncol.item()) == k
    assert st.tasks_popped == tasks
    assert st.hub_posts >= 1


@pytest.mark.parametrize("split", [8, 100])
@pytest.mark.parametrize("worker", [64, 1024])
def test_color_hub_board_concurrent(worker, split):
    """Many workers on split colouring tasks: the all-ordered colouring (unique
    whatever the schedule) equals the oracle, and default runs stay proper."""
    atos = _atos()
    for gi in (1, 2, 4, 5, 7):
        g = SMALL[gi]
        dg = _dev(g, int64=(gi % 2 == 0))
        cfg = atos.Config(worker=worker, fetch=min(worker, 64), split_degree=split,
                          color_order_degree=1, timeout_ms=20000)
        col, ncol, st = atos.color(dg, seed=5, cfg=cfg, stats=True)
        ref, k, _ = oracle.color_fifo(g, 5, order_degree=1)
        np.testing.assert_array_equal(col.cpu().numpy(), ref, err_msg=g.name)
        assert int(ncol.item()) == k
        assert st.hub_posts >= 1 or np.diff(g.offsets).max() <= split
        cfg.color_order_degree = 0
        col, ncol = atos.color(dg, seed=3, cfg=cfg)
        _check_gc(g, col, ncol, tight=False)


@pytest.mark.parametrize("gi", range(len(SMALL)), ids=[g.name for g in SMALL])
@pytest.mark.parametrize("worker,fetch", [(64, 8), (1024, 256)])
def test_discrete_rounds(gi, worker, fetch):
    """Discrete kernels (one launch per round over the same worklist): a round
    takes exactly the tasks published before it, so BFS takes one round per
    level; results match the oracle like the persistent kernel's."""
    import torch
    atos = _atos()
    g = SMALL[gi]
    dg = _dev(g, int64=(gi % 2 == 1))
    cfg = atos.Config(strategy=atos.DISCRETE, worker=worker, fetch=fetch, timeout_ms=20000)
    src = gg.max_degree_vertex(g)
    depth, st = atos.bfs(dg, src, cfg=cfg, stats=True)
    ref = oracle.bfs(g, src)
    np.testing.assert_array_equal(depth.cpu().numpy(), ref)
    assert st.rounds == ref.max() + 1
    res = torch.empty(g.n, dtype=torch.float32, device="cuda")
    rank, st = atos.pagerank(dg, D, EPS, cfg=cfg, residual=res, stats=True)
    _check_pr(g, rank, res)
    assert st.rounds >= 1
    col, ncol = atos.color(dg, seed=3, cfg=cfg)
    _check_gc(g, col, ncol, tight=False)


@pytest.mark.parametrize("gi", range(len(SMALL)), ids=[g.name for g in SMALL])
@pytest.mark.parametrize("tail", [1, 40, 1 << 30])
def test_discrete_tail_switch(gi, tail):
    """Discrete rounds until a round leaves at most `tail` tasks, then one
    persistent launch for the rest: the results are the persistent kernel's
    (exact BFS, bounded PageRank, valid colourings), and the switch comes no
    later than the pure discrete run's last round."""
    import torch
    atos = _atos()
    g = SMALL[gi]
    dg = _dev(g)
    src = gg.max_degree_vertex(g)
    ref = oracle.bfs(g, src)
    cfg = atos.Config(strategy=atos.DISCRETE, worker=256, fetch=16, discrete_tail=tail,
                      timeout_ms=20000)
    depth, st = atos.bfs(dg, src, cfg=cfg, stats=True)
    np.testing.assert_array_equal(depth.cpu().numpy(), ref)
    assert 1 <= st.rounds <= ref.max() + 1
    if tail >= g.n:
        assert st.rounds <= 2  # the first round leaves at most n tasks
    res = torch.empty(g.n, dtype=torch.float32, device="cuda")
    rank, st = atos.pagerank(dg, D, EPS, cfg=cfg, residual=res, stats=True)
    _check_pr(g, rank, res)
    col, ncol = atos.color(dg, seed=3, cfg=cfg)
    _check_gc(g, col, ncol, tight=False)


@pytest.mark.parametrize("gi", range(len(SMALL)), ids=[g.name for g in SMALL])
@pytest.mark.parametrize("worker,fetch", [(64, 8), (256, 64), (1024, 256)])
def test_rounds_in_one_launch(gi, worker, fetch):
    """Discrete rounds inside one persistent launch (the workers advance the
    round once its tasks are all taken): exact BFS, bounded PageRank, valid
    colourings; BFS needs at least one round per level after the source's."""
    import torch
    atos = _atos()
    g = SMALL[gi]
    dg = _dev(g, int64=(gi % 2 == 1))
    cfg = atos.Config(strategy=atos.ROUNDS, worker=worker, fetch=fetch, timeout_ms=20000)
    src = gg.max_degree_vertex(g)
    depth, st = atos.bfs(dg, src, cfg=cfg, stats=True)
    ref = oracle.bfs(g, src)
    np.testing.assert_array_equal(depth.cpu().numpy(), ref)
    assert st.rounds >= 1
    res = torch.empty(g.n, dtype=torch.float32, device="cuda")
    rank, st = atos.pagerank(dg, D, EPS, cfg=cfg, residual=res, stats=True)
    _check_pr(g, rank, res)
    col, ncol = atos.color(dg, seed=3, cfg=cfg)
    _check_gc(g, col, ncol, tight=False)


def test_rounds_single_worker_bfs_takes_one_round_per_level():
    """With one worker taking every task of a round at once, a round is a
    level: the round count is the BFS depth plus one, as for discrete
    launches."""
    atos = _atos()
    for g in (SMALL[0], SMALL[3], SMALL[6]):
        dg = _dev(g)
        src = gg.max_degree_vertex(g)
        ref = oracle.bfs(g, src)
        cfg = atos.Config(strategy=atos.ROUNDS, worker=1024, fetch=1024, grid=1,
                          queue_layout=atos.QUEUE_GLOBAL, timeout_ms=20000)
        depth, st = atos.bfs(dg, src, cfg=cfg, stats=True)
        np.testing.assert_array_equal(depth.cpu().numpy(), ref)
        assert st.rounds == ref.max() + 1, g.name


@pytest.mark.parametrize("gi", [2, 4, 5, 7], ids=[SMALL[i].name for i in (2, 4, 5, 7)])
def test_discrete_single_worker_colouring_equals_fifo_oracle(gi):
    """One worker taking one task at a time over discrete rounds still pops in
    FIFO order, so the colouring and its task count equal the oracle's."""
    atos = _atos()
    g = SMALL[gi]
    cfg = atos.Config(strategy=atos.DISCRETE, worker=64, fetch=1, grid=1,
                      queue_layout=atos.QUEUE_GLOBAL, color_order_degree=32)
    col, ncol, st = atos.color(_dev(g), seed=3, cfg=cfg, stats=True)
    ref, k, tasks = oracle.color_fifo(g, 3, order_degree=32)
    np.testing.assert_array_equal(col.cpu().numpy(), ref)
    assert st.tasks_popped == tasks


@pytest.mark.parametrize("policy", [0, 1, 2])
def test_fetch_policies_keep_results(policy):
    """Fixed claims, adaptive claims (a worker's share of a shallow ring) and
    the per-application default all give exact BFS, bounded PageRank, valid
    colourings and the unique all-ordered colouring."""
    import torch
    atos = _atos()
    for gi in (4, 5, 6):
        g = SMALL[gi]
        dg = _dev(g)
        cfg = atos.Config(worker=256, fetch=64, fetch_policy=policy, timeout_ms=20000)
        src = gg.max_degree_vertex(g)
        np.testing.assert_array_equal(atos.bfs(dg, src, cfg=cfg).cpu().numpy(), oracle.bfs(g, src))
        res = torch.empty(g.n, dtype=torch.float32, device="cuda")
        _check_pr(g, atos.pagerank(dg, D, EPS, cfg=cfg, residual=res), res)
        col, ncol = atos.color(dg, seed=3, cfg=cfg)
        _check_gc(g, col, ncol, tight=False)
        cfg.color_order_degree = 1
        col, _ = atos.color(dg, seed=5, cfg=cfg)
        np.testing.assert_array_equal(col.cpu().numpy(), oracle.color_fifo(g, 5, order_degree=1)[0])


@pytest.mark.parametrize("push", [1, 2])
@pytest.mark.parametrize("strategy", [0, 2])
def test_push_policies_keep_results(push, strategy):
    """Publishing into the worker's own XCD ring or into the shallowest ring,
    persistent or discrete: exact BFS, bounded PageRank, valid colourings and
    the unique all-ordered colouring."""
    import torch
    atos = _atos()
    for gi in (3, 5, 6):
        g = SMALL[gi]
        dg = _dev(g)
        cfg = atos.Config(strategy=strategy, worker=256, fetch=64, push_policy=push,
                          queue_layout=atos.QUEUE_PER_XCD, timeout_ms=20000)
        src = gg.max_degree_vertex(g)
        np.testing.assert_array_equal(atos.bfs(dg, src, cfg=cfg).cpu().numpy(), oracle.bfs(g, src))
        res = torch.empty(g.n, dtype=torch.float32, device="cuda")
        _check_pr(g, atos.pagerank(dg, D, EPS, cfg=cfg, residual=res), res)
        col, ncol = atos.color(dg, seed=3, cfg=cfg)
        _check_gc(g, col, ncol, tight=False)
        cfg.color_order_degree = 1
        col, _ = atos.color(dg, seed=5, cfg=cfg)
        np.testing.assert_array_equal(col.cpu().numpy(), oracle.color_fifo(g, 5, order_degree=1)[0])


def test_fetch_policy_rejects_unknown_values():
    atos = _atos()
    dg = _dev(SMALL[0])
    with pytest.raises(atos.AtosError):
        atos.bfs(dg, 0, cfg=atos.Config(fetch_policy=3))
    with pytest.raises(atos.AtosError):
        atos.bfs(dg, 0, cfg=atos.Config(push_policy=3))  # query rings are for the server only


def _double_star(leaves):
    """Two hubs joined by an edge, each with `leaves` leaves."""
    n = 2 + 2 * leaves
    src = [0] + [0] * leaves + [1] * leaves
    dst = [1] + list(range(2, 2 + leaves)) + list(range(2 + leaves, n))
    return gg.csr_from_edges(n, np.array(src), np.array(dst), f"dstar{leaves}")


@pytest.mark.parametrize("worker", [64, 256, 1024])
def test_hub_board_splits_high_degree_tasks(worker):
    """Tasks above the hub threshold are posted to the board and processed in
    chunks by all workers; results stay exact (BFS) / within bounds (PR).
    split_degree = -1 turns the board off, a small threshold posts many tasks."""
    import torch
    atos = _atos()
    for g in (gg.star_graph(20000), _double_star(40000)):
        dg = _dev(g)
        for split in (0, 300, -1):
            cfg = atos.Config(worker=worker, fetch=min(worker, 64), timeout_ms=20000,
                              split_degree=split)
            for s in (0, g.n - 1):
                depth, st = atos.bfs(dg, s, cfg=cfg, stats=True)
                np.testing.assert_array_equal(depth.cpu().numpy(), oracle.bfs(g, s))
                assert (st.hub_posts >= 1) == (split != -1)
            res = torch.empty(g.n, dtype=torch.float32, device="cuda")
            rank, st = atos.pagerank(dg, D, EPS, cfg=cfg, residual=res, stats=True)
            _check_pr(g, rank, res)
            assert (st.hub_posts >= 1) == (split != -1)


@pytest.mark.parametrize("gi", range(len(SMALL)), ids=[g.name for g in SMALL])
def test_small_split_degree_posts_many_hub_tasks(gi):
    """A threshold of 8 edges sends most tasks of the small graphs through the
    hub board (and its fallback when all probed entries are taken)."""
    import torch
    atos = _atos()
    g = SMALL[gi]
    dg = _dev(g, int64=(gi % 2 == 0))
    cfg = atos.Config(worker=64, fetch=16, split_degree=8, timeout_ms=20000)
    src = gg.max_degree_vertex(g) if g.n else 0
    if g.n:
        depth = atos.bfs(dg, src, cfg=cfg)
        np.testing.assert_array_equal(depth.cpu().numpy(), oracle.bfs(g, src))
    res = torch.empty(g.n, dtype=torch.float32, device="cuda")
    rank = atos.pagerank(dg, D, EPS, cfg=cfg, residual=res)
    _check_pr(g, rank, res)


@pytest.mark.parametrize("app", ["pagerank", "color"])
def test_autotune_strategies_keep_results(app):
    """The tuner's second stage (kernel strategy x push policy at the winning
    launch shape) runs every strategy on PageRank and colouring; the winner,
    whatever it is, gives a bounded PageRank or a valid colouring."""
    import torch
    atos = _atos()
    g = SMALL[6]
    dg = _dev(g)
    appc = atos.APP_PAGERANK if app == "pagerank" else atos.APP_COLOR
    best, table = atos.autotune(dg, appc, reps=1, base=atos.Config(timeout_ms=20000))
    stage2 = table[84:]
    assert len(stage2) == 6 and all(t["status"] == 0 for t in stage2), stage2
    assert {t["strategy"] for t in stage2} == {atos.PERSISTENT, atos.DISCRETE, atos.ROUNDS}
    if app == "pagerank":
        res = torch.empty(g.n, dtype=torch.float32, device="cuda")
        rank = atos.pagerank(dg, D, EPS, cfg=best, residual=res)
        _check_pr(g, rank, res)
    else:
        col, ncol = atos.color(dg, seed=3, cfg=best)
        _check_gc(g, col, ncol, tight=False)
