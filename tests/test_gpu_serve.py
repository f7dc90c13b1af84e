"""Serving daemon (continuous batching) through the C-ABI: every query result
matches the oracle, and is the same alone and in a mix of concurrent queries.

BFS depths are compared bit for bit.  Personalized PageRank (eps 1e-6, the
serving workload's accuracy) is held to the push method's one-sided bound
0 <= x - p <= deg * eps / (1 - d) against the FP64 oracle, to its mass
identity, and to residues <= eps; alone and in the mix both satisfy it, so
they differ by at most that bound.
"""
import time

import numpy as np
import pytest

import oracle
from oracle import checks
from paper_2112_00132_amd import graphgen as gg

pytestmark = pytest.mark.gpu

D = 0.85
D32 = float(np.float32(D))  # the damping the device computes with (an FP32 argument)
PPR_EPS = 1e-6
APP_BFS, APP_PR = 1, 2


def _atos():
    import paper_2112_00132_amd as atos
    return atos


def _graphs():
    return [gg.rmat_graph(12, 8, seed=21, permute_seed=4),
            gg.grid_graph(48, seed=22),
            gg.rmat_graph(10, 16, seed=23),
            gg.star_graph(3000)]


GRAPHS = _graphs()


def _dev_graphs(atos):
    return [atos.Graph.from_csr(g.offsets, g.cols, offsets_int64=(i % 2 == 0))
            for i, g in enumerate(GRAPHS)]


def _queries(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        gi = int(rng.integers(len(GRAPHS)))
        app = APP_BFS if rng.random() < 0.7 else APP_PR
        src = int(rng.integers(GRAPHS[gi].n))
        out.append((gi, app, src))
    return out


def _serve(srv, queries, limit_s=20.0):
    """Submit every query (retrying while the server has no room), collect
    every result; returns {index: (completion, result)}."""
    backlog = list(enumerate(queries))
    inflight, done = {}, {}
    t0 = time.time()
    reported = False
    while (backlog or inflight) and time.time() - t0 < limit_s:
        if not reported and time.time() - t0 > 5.0:  # slow: show where the queries stand
            reported = True
            snap = srv.snapshot()
            print("slow after 5 s: inflight", sorted(inflight.values()), "daemon",
                  {k: v for k, v in snap.items() if k != "rings"})
            for q, r in enumerate(snap["rings"]):
                if r["tail"] != r["head"]:
                    print("ring", q, r)
        while backlog:
            i, (gi, app, src) = backlog[0]
            qid = srv.submit(gi, app, src, damping=D, epsilon=PPR_EPS, tag=i)
            if qid is None:
                break
            inflight[qid] = i
            backlog.pop(0)
        for c in srv.poll():
            i = inflight.pop(c.query_id)
            assert c.tag == i
            assert c.status == 0
            done[i] = (c, srv.result(c))
            srv.release(c.query_id)
        time.sleep(0.0002)
    if inflight:  # report where the unfinished queries stand before the test fails
        print("unfinished queries", sorted(inflight), "after", round(time.time() - t0, 1), "s")
        snap = srv.snapshot()
        print("daemon", {k: snap[k] for k in ("status", "submit_head", "comp_tail", "active",
                                             "admitted", "completed", "timeout_after_s")})
        print("busy slots", snap["slots"])
        for q, r in enumerate(snap["rings"]):
            if r["tail"] != r["head"]:
                print("ring", q, r)
    return done


def _check_one(q, res, graphs=None):
    gi, app, src = q
    g = (graphs or GRAPHS)[gi]
    if app == APP_BFS:
        np.testing.assert_array_equal(res, oracle.bfs(g, src))
        return
    rank, residue = (r.astype(np.float64) for r in res)  # FP32 outputs
    assert residue.max(initial=0.0) <= float(np.float32(PPR_EPS))
    x, _, _, bound = oracle.ppr(g, src, D32)
    v = checks.pagerank_violations(g, rank, x, D32, PPR_EPS, rel_tol=None, ref_bound=bound)
    assert v == [], v
    obs, exp = checks.ppr_mass(g, src, rank, residue, D32)
    assert abs(obs - exp) <= 1e-6, (obs, exp)  # FP32 rounding of the outputs


def _cfg(atos, **kw):
    kw.setdefault("timeout_ms", 45000)
    return atos.ServerConfig(**kw)


@pytest.mark.parametrize("worker,fetch,layout,push", [(256, 64, 0, 0), (64, 16, 2, 1), (1024, 128, 2, 3),
                                                     (1024, 256, 2, 2), (256, 256, 2, 3)])
def test_mix_matches_oracle_and_alone(worker, fetch, layout, push):
    """Every ring layout: one shared ring; per-XCD rings with pushes to the own
    ring, to the shallowest ring, or to the ring of each task's query."""
    atos = _atos()
    dgs = _dev_graphs(atos)
    srv = atos.Server(dgs, arena_bytes=256 << 20,
                      cfg=_cfg(atos, worker=worker, fetch=fetch, max_queries=32, queue_layout=layout,
                               push_policy=push))
    qs = _queries(48, seed=worker)
    srv.start()
    try:
        mix = _serve(srv, qs)
        assert len(mix) == len(qs), f"{len(qs) - len(mix)} queries unfinished"
        alone = {}
        for i, q in enumerate(qs[:16]):
            alone.update({i: r for r in _serve(srv, [q]).values()})
    finally:
        st = srv.stop()
    assert st.status == 0
    assert st.rounds == len(qs) + 16
    assert len(mix) == len(qs)
    for i, q in enumerate(qs):
        _check_one(q, mix[i][1])
    for i in alone:
        gi, app, _ = qs[i]
        if app == APP_BFS:
            np.testing.assert_array_equal(alone[i][1], mix[i][1])
        else:
            deg = np.diff(GRAPHS[gi].offsets).astype(np.float64)
            diff = np.abs(alone[i][1][0].astype(np.float64) - mix[i][1][0].astype(np.float64))
            assert np.all(diff <= deg * PPR_EPS / (1 - D32) + 2e-7)
    srv.close()


def test_admission_waits_for_memory_and_slots():
    """An arena with room for a few query states and 3 slots: most submits
    are refused at first (EAGAIN) and admitted as earlier queries release."""
    atos = _atos()
    dgs = _dev_graphs(atos)
    c = _cfg(atos, max_queries=3)
    heap = 16 * max(g.n for g in GRAPHS) * 2 + (2 << 20)  # about two PageRank states
    srv = atos.Server(dgs, arena_bytes=atos.server_arena_bytes(dgs, c) + heap, cfg=c)
    qs = _queries(30, seed=5)
    srv.start()
    try:
        got = _serve(srv, qs)
    finally:
        st = srv.stop()
    assert st.status == 0
    assert len(got) == len(qs)
    for i, q in enumerate(qs):
        _check_one(q, got[i][1])
    srv.close()


def test_restart_and_bad_submissions():
    atos = _atos()
    dgs = _dev_graphs(atos)
    srv = atos.Server(dgs, arena_bytes=128 << 20, cfg=_cfg(atos, max_queries=8))
    with pytest.raises(atos.AtosError):
        srv.submit(0, APP_BFS, 0)  # not running
    for rnd in range(2):
        srv.start()
        try:
            with pytest.raises(atos.AtosError):
                srv.submit(len(GRAPHS), APP_BFS, 0)  # no such graph
            with pytest.raises(atos.AtosError):
                srv.submit(0, APP_BFS, GRAPHS[0].n)  # source out of range
            with pytest.raises(atos.AtosError):
                srv.submit(0, 3, 0)  # colouring is not served
            with pytest.raises(atos.AtosError):
                srv.submit(0, APP_PR, 0, damping=1.5)
            qs = _queries(6, seed=40 + rnd)
            got = _serve(srv, qs)
            snap = srv.snapshot()
            if snap["status"] != 0:
                print("daemon", {k: v for k, v in snap.items() if k != "rings"})
            assert snap["status"] == 0 and snap["active"] == 0 and snap["slots"] == {}
            assert snap["admitted"] == snap["completed"] == len(qs)
            assert all(r["head"] <= r["tail"] for r in snap["rings"])
        finally:
            st = srv.stop()
        assert st.status == 0 and st.rounds == len(qs)
        for i, q in enumerate(qs):
            _check_one(q, got[i][1])
    with pytest.raises(atos.AtosError):
        srv.submit(0, APP_BFS, 0)  # stopped
    srv.close()


def test_single_query_ppr_entry_point():
    """atos_ppr (one launch per query, the serving baseline) meets the same bound."""
    import torch
    atos = _atos()
    for gi, g in enumerate(GRAPHS):
        dg = atos.Graph.from_csr(g.offsets, g.cols)
        for src in (gg.max_degree_vertex(g), 0, g.n - 1):
            res = torch.empty(g.n, dtype=torch.float32, device="cuda")
            for strategy in (atos.PERSISTENT, atos.BSP):
                rank = atos.ppr(dg, src, D, PPR_EPS, cfg=atos.Config(strategy=strategy), residual=res)
                r = rank.cpu().numpy().astype(np.float64)
                assert res.max().item() <= float(np.float32(PPR_EPS))
                x, _, _, bound = oracle.ppr(g, src, D32)
                v = checks.pagerank_violations(g, r, x, D32, float(np.float32(PPR_EPS)), rel_tol=None,
                                               ref_bound=bound)
                assert v == [], (g.name, src, strategy, v)


# Graphs above one 16,384-vertex chunk of the daemon's state initialisation
# and result copy, so every query's init and final steps span several chunks
# (int32 offsets on the R-MAT, int64 on the grid), as on the serving graphs.
BIG = [gg.rmat_graph(16, 8, seed=31, permute_seed=2), gg.grid_graph(256, diag_frac=0.0, seed=32)]


def test_multichunk_queries_match_oracle_and_alone():
    atos = _atos()
    assert all(g.n > 2 * 16384 for g in BIG)
    dgs = [atos.Graph.from_csr(BIG[0].offsets, BIG[0].cols, offsets_int64=False),
           atos.Graph.from_csr(BIG[1].offsets, BIG[1].cols, offsets_int64=True)]
    rng = np.random.default_rng(33)
    qs = []
    for i in range(24):
        gi = i % 2
        app = APP_BFS if rng.random() < 0.6 else APP_PR
        src = int(gg.random_nonisolated_sources(BIG[gi], 1, seed=100 + i)[0])
        qs.append((gi, app, src))
    qs.append((0, APP_BFS, int(np.flatnonzero(np.diff(BIG[0].offsets) == 0)[0])))  # isolated source
    srv = atos.Server(dgs, arena_bytes=512 << 20, cfg=_cfg(atos, max_queries=16))
    srv.start()
    try:
        print(f"multichunk: {len(qs)} queries on n={[g.n for g in BIG]}", flush=True)
        mix = _serve(srv, qs, limit_s=40.0)
        assert len(mix) == len(qs), f"{len(qs) - len(mix)} queries unfinished"
        alone = {}
        for i in (0, 1, 2, 3, 5, 7):
            alone.update({i: r for r in _serve(srv, [qs[i]], limit_s=20.0).values()})
    finally:
        st = srv.stop()
    assert st.status == 0
    for i, q in enumerate(qs):
        _check_one(q, mix[i][1], BIG)
        assert mix[i][0].tasks > (BIG[q[0]].n + 16383) // 16384  # init chunks + the source task
    for i, (c, res) in alone.items():
        gi, app, _ = qs[i]
        if app == APP_BFS:
            np.testing.assert_array_equal(res, mix[i][1])
        else:
            deg = np.diff(BIG[gi].offsets).astype(np.float64)
            diff = np.abs(res[0].astype(np.float64) - mix[i][1][0].astype(np.float64))
            assert np.all(diff <= deg * PPR_EPS / (1 - D32) + 2e-7)
    srv.close()
