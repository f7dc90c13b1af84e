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
