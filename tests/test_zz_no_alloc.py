"""atos_bfs_noalloc (the BFS entry point that allocates nothing) against atos_bfs.

Both are called through the C ABI on the same device graph; the depths must
be bit-identical, and equal to the oracle's, on two calls in a row, the second
on a smaller graph (so the fixed scratch keeps the first call's contents and
the second call must not be misled by them).  Sizes beyond the scratch are
refused on the host before anything is enqueued."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2112_00132_amd import graphgen as gg

pytestmark = pytest.mark.gpu

ENOMEM = 2


def _lib():
    import paper_2112_00132_amd as atos
    return atos._load()


def _call_noalloc(dg, src, out, cfg=None):
    import paper_2112_00132_amd as atos
    c = (cfg or atos.Config())._c()
    st = atos._Stats()
    rc = _lib().atos_bfs_noalloc(dg._h, ctypes.c_int64(int(src)), atos._ptr(out), ctypes.byref(c),
                                 atos._stream_handle(None), ctypes.byref(st))
    return rc, st


def _call_with_workspace(dg, src, out, cfg=None):
    import paper_2112_00132_amd as atos
    cfg = cfg or atos.Config()
    ws = dg.workspace(atos.APP_BFS, cfg)
    c = cfg._c()
    st = atos._Stats()
    rc = _lib().atos_bfs(dg._h, ctypes.c_int64(int(src)), atos._ptr(out), atos._ptr(ws), ws.numel(),
                         ctypes.byref(c), atos._stream_handle(None), ctypes.byref(st))
    return rc, st


CASES = [
    # (graph, int64 offsets, launch shape): the larger graph first
    (lambda: gg.rmat_graph(15, 8, seed=11, permute_seed=2), False, dict(worker=1024, fetch=256)),
    (lambda: gg.grid_graph(48, seed=12), True, dict(worker=256, fetch=64)),
]


def test_noalloc_matches_workspace_entry_point_twice():
    import torch
    import paper_2112_00132_amd as atos
    for make, i64, shape in CASES:
        g = make()
        dg = atos.Graph.from_csr(g.offsets, g.cols, offsets_int64=i64)
        cfg = atos.Config(timeout_ms=20000, **shape)
        for src in (gg.max_degree_vertex(g), g.n - 1):
            print(f"noalloc: {g.name} n={g.n} src={src} {shape}", flush=True)
            a = torch.full((g.n,), 7, dtype=torch.int32, device="cuda")
            b = torch.full((g.n,), 9, dtype=torch.int32, device="cuda")
            rc, st = _call_noalloc(dg, src, a, cfg)
            assert rc == 0 and st.status == 0, (rc, st.status)
            assert st.device_ms == 0.0 and st.kernel_ms == 0.0  # no events on this path
            rc, st2 = _call_with_workspace(dg, src, b, cfg)
            assert rc == 0 and st2.status == 0, (rc, st2.status)
            da, db = a.cpu().numpy(), b.cpu().numpy()
            np.testing.assert_array_equal(da, db)
            np.testing.assert_array_equal(da, oracle.bfs(g, src))
            assert st.tasks_popped >= int((da >= 0).sum())


def test_noalloc_default_config_and_binding():
    import paper_2112_00132_amd as atos
    g = gg.path_graph(3000)
    dg = atos.Graph.from_csr(g.offsets, g.cols, offsets_int64=False)
    d = atos.bfs_noalloc(dg, 17).cpu().numpy()
    np.testing.assert_array_equal(d, oracle.bfs(g, 17))
    d2, st = atos.bfs_noalloc(dg, 0, stats=True)
    np.testing.assert_array_equal(d2.cpu().numpy(), oracle.bfs(g, 0))
    assert st.status == 0


def test_noalloc_refuses_a_workspace_beyond_the_scratch():
    import torch
    import paper_2112_00132_amd as atos
    g = gg.path_graph(100)
    dg = atos.Graph.from_csr(g.offsets, g.cols)
    big = atos.Config(queue_capacity=1 << 24)  # 8 rings x 2^24 x 8 B = 1 GiB of rings
    assert dg.workspace_bytes(atos.APP_BFS, big) > atos.NOALLOC_SCRATCH_BYTES
    out = torch.full((g.n,), 5, dtype=torch.int32, device="cuda")
    rc, _ = _call_noalloc(dg, 0, out, big)
    assert rc == ENOMEM
    torch.cuda.synchronize()
    assert int(out.min()) == 5 and int(out.max()) == 5  # nothing was enqueued
    # the refusal left the scratch usable
    d = atos.bfs_noalloc(dg, 3).cpu().numpy()
    np.testing.assert_array_equal(d, oracle.bfs(g, 3))
