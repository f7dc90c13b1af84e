"""Batched runs: many BFS and PageRank instances in one persistent launch.

Every instance must equal its own oracle (BFS bit-exact, PageRank within
the stated bound) and its alone-run through atos_bfs / atos_pagerank (BFS
bit-identical; PageRank both within the bound).  hipGraph replays must
reproduce the eager result on every replay."""
import types

import numpy as np
import pytest

import oracle
from oracle import checks
from paper_2112_00132_amd import graphgen as gg

pytestmark = pytest.mark.gpu

D = 0.85
EPS = 1e-7


def _host_graph(o, c):
    o = o.cpu().numpy().astype(np.int64)
    return types.SimpleNamespace(n=o.size - 1, offsets=o, cols=c.cpu().numpy().astype(np.int32))


@pytest.fixture(scope="module")
def small_batch():
    import torch
    import paper_2112_00132_amd as atos
    w = gg.batch_workload(n_graphs=24, n_pagerank=6, scales=(6, 10), edge_factors=(4, 32),
                          grid_sides=(8, 40), seed=4)
    dg = atos.Graph(w.offsets.cuda(), w.cols.cuda())
    return w, dg


def _check_instance(atos, k, w, state, res, alone=True):
    import torch
    app, vb, ve, src = w.instances[k]
    o, c, lsrc = w.local[k]
    hg = _host_graph(o, c)
    if app == atos.APP_BFS:
        got = state[vb:ve].cpu().numpy()
        ref = oracle.bfs(hg, lsrc)
        np.testing.assert_array_equal(got, ref, err_msg=f"instance {k} {w.kinds[k]}")
        if alone:
            lg = atos.Graph(o.cuda(), c.cuda())
            np.testing.assert_array_equal(atos.bfs(lg, lsrc).cpu().numpy(), got)
        return 0.0
    rank = state[vb:ve].view(torch.float32).cpu().numpy().astype(np.float64)
    r = res[vb:ve].cpu().numpy().astype(np.float64)
    x, _, _, bound = oracle.pagerank(hg, D)
    assert r.max(initial=0.0) <= float(np.float32(EPS))
    v = checks.pagerank_violations(hg, rank, x, D, EPS, ref_bound=bound)
    assert v == [], (k, w.kinds[k], v)
    if not alone:
        return 0.0
    lg = atos.Graph(o.cuda(), c.cuda())
    lres = torch.empty(lg.n, dtype=torch.float32, device="cuda")
    lrank = atos.pagerank(lg, D, EPS, residual=lres).cpu().numpy().astype(np.float64)
    assert checks.pagerank_violations(hg, lrank, x, D, EPS, ref_bound=bound) == []
    return float(np.abs(lrank - rank).max(initial=0.0))


def test_batch_instances_match_oracle_and_alone_runs(small_batch):
    import torch
    import paper_2112_00132_amd as atos
    w, dg = small_batch
    b = atos.Batch(dg, w.instances, D, EPS)
    res = torch.zeros(w.n, dtype=torch.float32, device="cuda")
    state, st = b.run(residual=res, stats=True)
    assert st.tasks_popped > 0
    worst = max(_check_instance(atos, k, w, state, res) for k in range(len(w.instances)))
    print(f"max |batched - alone| PageRank difference: {worst:.3g}")


@pytest.mark.parametrize("worker,fetch,layout", [(64, 8, 0), (1024, 256, 0), (256, 64, 3),
                                                 (1024, 256, 3)])
def test_batch_other_worker_sizes(small_batch, worker, fetch, layout):
    """Other launch shapes, and the segmented layout (every task in the ring of
    its instance's segment)."""
    import torch
    import paper_2112_00132_amd as atos
    w, dg = small_batch
    b = atos.Batch(dg, w.instances, D, EPS,
                   cfg=atos.Config(worker=worker, fetch=fetch, queue_layout=layout))
    res = torch.zeros(w.n, dtype=torch.float32, device="cuda")
    state = b.run(residual=res)
    for k in range(len(w.instances)):
        _check_instance(atos, k, w, state, res, alone=False)


def _pr_combinable(atos, w):
    """Whether a PageRank instance has a vertex of degree >= 64 (combinable)."""
    for k, (app, _, _, _) in enumerate(w.instances):
        if app == atos.APP_PAGERANK:
            o = w.local[k][0].cpu().numpy()
            if (np.diff(o) >= 64).any():
                return True
    return False


@pytest.mark.parametrize("comb", [-1, 1, 4096])
def test_batch_residue_combining(small_batch, comb):
    """Residue combining of the PageRank instances (BFS instances are not
    touched): off, flushed after every batch of tasks, and with a small
    window, every instance meets its oracle; the counters account for it;
    set_config switches it on the same workspace."""
    import torch
    import paper_2112_00132_amd as atos
    w, dg = small_batch
    can = _pr_combinable(atos, w)
    b = atos.Batch(dg, w.instances, D, EPS, cfg=atos.Config(worker=1024, fetch=256, pr_combine=comb))
    for step in (comb, 4096 if comb < 0 else -1):
        b.set_config(atos.Config(worker=1024, fetch=256, pr_combine=step))
        res = torch.zeros(w.n, dtype=torch.float32, device="cuda")
        state, st = b.run(residual=res, stats=True)
        for k in range(len(w.instances)):
            _check_instance(atos, k, w, state, res, alone=False)
        if step < 0 or not can:
            assert st.combined_updates == 0 and st.combine_atomics == 0
        else:
            assert 0 < st.combine_atomics <= st.combined_updates < st.edges_scanned


@pytest.mark.parametrize("layout", [0, 3])
def test_batch_graph_replays_match_eager(small_batch, layout):
    import torch
    import paper_2112_00132_amd as atos
    w, dg = small_batch
    b = atos.Batch(dg, w.instances, D, EPS, cfg=atos.Config(queue_layout=layout))
    res_e = torch.zeros(w.n, dtype=torch.float32, device="cuda")
    eager = b.run(residual=res_e).clone()
    stream = torch.cuda.Stream()
    state = torch.zeros(w.n, dtype=torch.int32, device="cuda")
    res = torch.zeros(w.n, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    ex = b.capture(state, res, stream=stream)
    bfs_mask = torch.zeros(w.n, dtype=torch.bool, device="cuda")
    for app, vb, ve, _ in w.instances:
        if app == atos.APP_BFS:
            bfs_mask[vb:ve] = True
    for replay in range(3):
        state.fill_(7)
        torch.cuda.synchronize()
        ex.launch(stream=stream)
        stream.synchronize()
        st = b.last_stats()
        assert st.status == 0
        assert torch.equal(state[bfs_mask], eager[bfs_mask]), f"replay {replay}"
        for k in range(len(w.instances)):
            _check_instance(atos, k, w, state, res, alone=False)
        # eager work between replays
        _ = atos.bfs(dg, w.instances[0][3])
        torch.cuda.synchronize()
    ex.close()


def test_batch_plan_rejects_bad_instances(small_batch):
    import paper_2112_00132_amd as atos
    w, dg = small_batch
    inst = list(w.instances)
    with pytest.raises(atos.AtosError):
        atos.Batch(dg, [inst[1], inst[0]] + inst[2:], D, EPS)  # not sorted by vertex_begin
    # an instance range that cuts a graph in two: its edges leave the range
    app, vb, ve, src = inst[0]
    cut = [(1, vb, vb + (ve - vb) // 2, vb)] + inst[1:]
    with pytest.raises(atos.AtosError) as e:
        atos.Batch(dg, cut, D, EPS)
    assert e.value.status == 1
    with pytest.raises(atos.AtosError):
        atos.Batch(dg, [(1, vb, ve, ve)] + inst[1:], D, EPS)  # source outside its range
    with pytest.raises(atos.AtosError):
        atos.Batch(dg, [(9, vb, ve, src)] + inst[1:], D, EPS)  # unknown application


def test_autotune_single_and_batch(small_batch, tmp_path):
    """The tuner sweeps the lower triangle of worker x fetch, then the kernel
    strategies and push policies at the winning shape; its winner is the
    fastest point of its own table, and runs with the winner stay exact."""
    import json
    import paper_2112_00132_amd as atos
    g = gg.rmat_graph(12, 16, seed=4, permute_seed=2)
    dg = atos.Graph.from_csr(g.offsets, g.cols)
    src = gg.max_degree_vertex(g)
    cache = str(tmp_path / "tune.json")
    calls = []
    best, table = atos.autotune(dg, atos.APP_BFS, source=src, reps=2, cache=cache,
                                progress=lambda d, t, r: calls.append((d, t, r)))
    # fetch powers of two up to min(worker, 256), 2 layouts; then 3 strategies x 2 push policies
    assert len(table) == 2 * (7 + 8 + 9 + 9 + 9) + 6
    # one progress call per point, in order, with that point's row of the table
    assert [c[0] for c in calls] == list(range(1, len(table) + 1))
    assert calls[-1][1] == len(table) and calls[0][1] == 84
    assert [c[2] for c in calls] == table
    assert all(t["fetch"] <= t["worker"] for t in table)
    stage1 = [t for t in table[:84] if t["status"] == 0]
    won = min(stage1, key=lambda t: t["median_ms"])
    stage2 = table[84:]
    assert sorted((t["strategy"], t["push_policy"]) for t in stage2) == [
        (s, p) for s in (atos.PERSISTENT, atos.DISCRETE, atos.ROUNDS) for p in (1, 2)]
    assert all((t["worker"], t["fetch"], t["queue_layout"]) ==
               (won["worker"], won["fetch"], won["queue_layout"]) for t in stage2)
    ok = [t for t in table if t["status"] == 0]
    fastest = min(ok, key=lambda t: t["median_ms"])
    assert (best.strategy, best.worker, best.fetch, best.push_policy) == \
        (fastest["strategy"], fastest["worker"], fastest["fetch"], fastest["push_policy"])
    np.testing.assert_array_equal(atos.bfs(dg, src, cfg=best).cpu().numpy(), oracle.bfs(g, src))
    with open(cache) as f:
        assert atos.tune_key(dg, atos.APP_BFS) in json.load(f)
    again, _ = atos.autotune(dg, atos.APP_BFS, source=src, cache=cache)  # served from the cache
    assert (again.worker, again.fetch) == (best.worker, best.fetch)

    w, dgb = small_batch
    b = atos.Batch(dgb, w.instances, D, EPS)
    bbest, btable = b.autotune(reps=1)
    # a batch also sweeps the segmented layout: 3 x 42 points, then 2 push policies
    assert bbest.worker in (64, 128, 256, 512, 1024) and len(btable) == 126 + 2
    assert {t["queue_layout"] for t in btable[:126]} == {1, 2, 3}
    assert bbest.strategy == atos.PERSISTENT
    b.set_config(bbest)
    import torch
    res = torch.zeros(w.n, dtype=torch.float32, device="cuda")
    state = b.run(residual=res)
    for k in range(len(w.instances)):
        _check_instance(atos, k, w, state, res, alone=False)
