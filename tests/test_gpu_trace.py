"""Per-batch trace of the persistent worker kernel (atos_trace_attach): the
records account for every task and edge the run's statistics count, hub
chunks name their hub, results are unchanged while tracing, and a full
buffer keeps counting without storing."""
import numpy as np
import pytest

import oracle
from paper_2112_00132_amd import graphgen as gg

pytestmark = pytest.mark.gpu


def _atos():
    import paper_2112_00132_amd as atos
    return atos


@pytest.mark.parametrize("split", [-1, 300])  # -1: hub board off
def test_trace_accounts_for_every_task_and_edge(split):
    atos = _atos()
    for g in (gg.star_graph(20000), gg.rmat_graph(12, 16, seed=4, permute_seed=2)):
        dg = atos.Graph.from_csr(g.offsets, g.cols)
        cfg = atos.Config(worker=256, fetch=64, split_degree=split, timeout_ms=20000)
        src = gg.max_degree_vertex(g)
        with atos.Trace(records=1 << 16) as tr:
            depth, st = atos.bfs(dg, src, cfg=cfg, stats=True)
        np.testing.assert_array_equal(depth.cpu().numpy(), oracle.bfs(g, src))
        r = tr.records()
        assert tr.count() == r.size > 0
        hub = (r["tasks"] & atos.TRACE_HUB_CHUNK) != 0
        assert int(r["tasks"][~hub].sum()) == st.tasks_popped
        assert int(r["edges"].astype(np.int64).sum()) == st.edges_scanned
        assert np.all(r["t_end"] >= r["t_begin"])
        assert np.all(r["vertex"] < g.n)
        deg = np.diff(g.offsets)
        if split > 0:
            assert hub.sum() >= 1 and st.hub_posts >= 1
            assert np.all(deg[r["vertex"][hub]] > split)
            assert np.all(r["tasks"][hub] == (atos.TRACE_HUB_CHUNK | 1))
        else:
            assert hub.sum() == 0
        # a batch's vertex is its highest-degree task: never above the graph's maximum
        assert deg[r["vertex"]].max() <= deg.max()
        # one batch holds at most FETCH tasks
        assert r["tasks"][~hub].max() <= 64
        # the clock rate is recorded, and the trace spans about the kernel's time
        assert 50_000 <= tr.clock_khz() <= 200_000
        tl = tr.timeline(bins=10)
        assert len(tl["gteps"]) == 10
        assert tl["span_ms"] <= st.kernel_ms * 1.05 + 0.05
        # (the timeline rounds its rates to 3 decimals)
        assert abs(sum(tl["gteps"]) * 1e9 * tl["ms"][0] * 2e-3 - st.edges_scanned) <= 0.02 * st.edges_scanned + 1


def test_trace_full_buffer_counts_without_storing_and_detach_stops():
    atos = _atos()
    g = gg.rmat_graph(12, 16, seed=4, permute_seed=2)
    dg = atos.Graph.from_csr(g.offsets, g.cols)
    cfg = atos.Config(worker=64, fetch=4, timeout_ms=20000)
    tr = atos.Trace(records=4).attach()
    try:
        atos.bfs(dg, 0, cfg=cfg)
    finally:
        tr.detach()
    n = tr.count()
    assert n > 4 and tr.records().size == 4
    atos.bfs(dg, 0, cfg=cfg)  # detached: nothing more is recorded
    assert tr.count() == n


def test_trace_rejects_bad_buffers():
    import torch
    atos = _atos()
    buf = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    lib = atos._load()
    assert lib.atos_trace_attach(buf.data_ptr(), 64) != 0  # too small
    assert lib.atos_trace_attach(buf.data_ptr() + 8, 1024) != 0  # misaligned
    host = np.zeros(4096, dtype=np.uint8)
    assert lib.atos_trace_attach(host.ctypes.data, 4096) != 0  # not device memory
    assert lib.atos_trace_attach(None, 0) == 0


@pytest.mark.parametrize("app", ["bfs", "pagerank", "color"])
def test_bsp_level_records(app):
    """A traced level-synchronous run records one entry per level plus its end:
    for BFS the frontier of level d is exactly the oracle's vertices at depth
    d, and the edges of a level are the degrees of its frontier; for every app
    the levels match stats.rounds and their edges sum to stats.edges_scanned.
    Tracing changes no result."""
    import torch
    atos = _atos()
    g = gg.grid_graph(48, seed=7)
    dg = atos.Graph.from_csr(g.offsets, g.cols)
    cfg = atos.Config(strategy=atos.BSP, worker=256)
    src = gg.max_degree_vertex(g)
    with atos.Trace(records=1 << 14) as tr:
        if app == "bfs":
            out, st = atos.bfs(dg, src, cfg=cfg, stats=True)
        elif app == "pagerank":
            out, st = atos.pagerank(dg, 0.85, 1e-7, cfg=cfg, stats=True)
        else:
            out, _, st = atos.color(dg, 3, cfg=cfg, stats=True)
        torch.cuda.synchronize()
    lv = tr.levels()
    assert lv["level"] == list(range(st.rounds))
    assert sum(lv["edges"]) == st.edges_scanned
    assert all(u >= 0 for u in lv["us"])
    assert tr.timeline()["ms"] == []  # no worker-batch records in a BSP run
    if app == "bfs":
        ref = oracle.bfs(g, src)
        np.testing.assert_array_equal(out.cpu().numpy(), ref)
        sizes = np.bincount(ref[ref >= 0])
        assert lv["frontier"] == sizes.tolist()
        deg = np.diff(g.offsets)
        assert lv["edges"] == [int(deg[ref == d].sum()) for d in range(len(sizes))]


@pytest.mark.parametrize("worker,one_per_cu", [(512, True), (1024, True), (256, False)])
def test_colouring_launches_one_worker_per_cu(worker, one_per_cu):
    """Colouring with 512- or 1024-thread workers launches one worker per CU
    whatever the register count would allow (its ordered chain only gets
    slower with more workers); smaller workers fill the CUs.  The trace names
    the worker of every batch."""
    import torch
    import paper_2112_00132_amd as atos
    g = gg.rmat_graph(14, 16, seed=5)
    dg = atos.Graph.from_csr(g.offsets, g.cols)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    with atos.Trace(records=1 << 20) as tr:
        atos.color(dg, 3, cfg=atos.Config(worker=worker, timeout_ms=20000))
        torch.cuda.synchronize()
    workers = tr.records()["worker"]
    assert workers.size > 0
    if one_per_cu:
        assert int(workers.max()) < n_cu
    else:
        assert int(workers.max()) >= n_cu  # more than one 256-thread worker per CU
