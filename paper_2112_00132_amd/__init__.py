"""Atos on MI355X: a persistent-worklist graph engine for gfx950.

Thin ctypes binding over ``libatos.so`` (C ABI declared in include/atos.h).
This module only marshals arguments: device memory comes from torch tensors,
streams from ``torch.cuda`` and every step of the computation runs in the
library's HIP kernels.  There is no CPU fallback: importing the compute
functions without a built library raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

__all__ = [
    "AtosError", "Config", "Stats", "Graph", "Batch", "Exec", "bfs", "bfs_noalloc", "pagerank",
    "ppr", "color",
    "autotune", "library_path",
    "PERSISTENT", "BSP", "DISCRETE", "ROUNDS", "APP_BFS", "APP_PAGERANK", "APP_COLOR",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_build", "libatos.so")

PERSISTENT = 0
BSP = 1
DISCRETE = 2
ROUNDS = 3  # discrete rounds inside one persistent launch
QUEUE_AUTO = 0
QUEUE_GLOBAL = 1
QUEUE_PER_XCD = 2
QUEUE_SEGMENTED = 3  # batches: every task into the ring of its vertex's segment of whole instances
PUSH_AUTO = 0
PUSH_OWN = 1
PUSH_SHALLOWEST = 2
PUSH_QUERY = 3
FETCH_AUTO = 0
FETCH_FIXED = 1
FETCH_ADAPTIVE = 2
APP_BFS = 1
APP_PAGERANK = 2
APP_COLOR = 3
GRAPH_SYMMETRIC = 1
GRAPH_VALIDATE = 2
_WS_HEADER_BYTES = 4096

_STATUS = {0: "ok", 1: "EINVAL", 2: "ENOMEM", 3: "EOVERFLOW", 4: "ETIMEOUT", 5: "EABORTED",
           6: "EHIP", 7: "ENOTSYMMETRIC", 8: "EUNSUPPORTED", 9: "EAGAIN"}
EAGAIN = 9


class AtosError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = int(status)
        super().__init__(f"{where}: {_STATUS.get(self.status, self.status)}")


class _Config(ctypes.Structure):
    _fields_ = [("strategy", ctypes.c_int32), ("worker", ctypes.c_int32),
                ("fetch", ctypes.c_int32), ("queue_layout", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("pr_check_size", ctypes.c_int32),
                ("queue_capacity", ctypes.c_int64), ("timeout_ms", ctypes.c_uint32),
                ("split_degree", ctypes.c_int32), ("color_order_degree", ctypes.c_int32),
                ("fetch_policy", ctypes.c_int32), ("push_policy", ctypes.c_int32),
                ("discrete_tail", ctypes.c_uint32), ("color_forbid_all", ctypes.c_int32),
                ("pr_combine", ctypes.c_int32), ("abort_flag", ctypes.c_void_p)]


class _BatchInstance(ctypes.Structure):
    _fields_ = [("app", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("vertex_begin", ctypes.c_int64), ("vertex_end", ctypes.c_int64),
                ("source", ctypes.c_int64)]


class _TuneResult(ctypes.Structure):
    _fields_ = [("cfg", _Config), ("median_ms", ctypes.c_float), ("status", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class _ServerConfig(ctypes.Structure):
    _fields_ = [("worker", ctypes.c_int32), ("fetch", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("max_queries", ctypes.c_int32), ("queue_capacity", ctypes.c_int64),
                ("timeout_ms", ctypes.c_uint32), ("queue_layout", ctypes.c_int32),
                ("push_policy", ctypes.c_int32), ("reserved", ctypes.c_uint32 * 3)]


class _Query(ctypes.Structure):
    _fields_ = [("graph", ctypes.c_int32), ("app", ctypes.c_int32), ("source", ctypes.c_int64),
                ("damping", ctypes.c_float), ("epsilon", ctypes.c_float), ("tag", ctypes.c_uint64),
                ("out", ctypes.c_void_p)]


class _Completion(ctypes.Structure):
    _fields_ = [("query_id", ctypes.c_uint64), ("tag", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("app", ctypes.c_int32), ("graph", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("state_offset", ctypes.c_uint64), ("tasks", ctypes.c_uint64),
                ("edges", ctypes.c_uint64), ("device_us", ctypes.c_double)]


class _Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("tasks_popped", ctypes.c_uint64), ("tasks_pushed", ctypes.c_uint64),
                ("edges_scanned", ctypes.c_uint64), ("rounds", ctypes.c_uint64),
                ("device_ms", ctypes.c_float), ("kernel_ms", ctypes.c_float),
                ("push_retries", ctypes.c_uint64), ("idle_iterations", ctypes.c_uint64),
                ("steals", ctypes.c_uint64), ("hub_posts", ctypes.c_uint64),
                ("combined_updates", ctypes.c_uint64), ("combine_atomics", ctypes.c_uint64)]


@dataclass
class Config:
    """Launch configuration (mirrors ``atos_config``; 0 = library default)."""
    strategy: int = PERSISTENT  # PERSISTENT, DISCRETE (a launch per round), ROUNDS or BSP
    worker: int = 0
    fetch: int = 0
    queue_layout: int = QUEUE_AUTO
    grid: int = 0
    pr_check_size: int = 0
    queue_capacity: int = 0
    timeout_ms: int = 0
    split_degree: int = 0  # hub-board threshold; 0 = default, -1 = never split
    color_order_degree: int = 0  # colouring ordered-class degree; 0 = default (8), -1 = none, -2 = ~sqrt(n) top-degree
    fetch_policy: int = 0  # FETCH_AUTO, FETCH_FIXED (up to `fetch`) or FETCH_ADAPTIVE (a share)
    push_policy: int = 0  # PUSH_AUTO, PUSH_OWN (own XCD's ring) or PUSH_SHALLOWEST
    discrete_tail: int = 0  # DISCRETE: queued tasks at which the rest runs persistent; 0 = never
    color_forbid_all: int = 0  # colouring: 1 = avoid every neighbour's colour (Alg 5/6 as printed)
    pr_combine: int = 0  # PageRank high-degree residue combining in LDS: N = flush window, -1 = off, 0 = default
    abort: "AbortFlag | None" = None  # host flag that stops the run (EABORTED) when set

    def _c(self) -> _Config:
        c = _Config()
        for f in ("strategy", "worker", "fetch", "queue_layout", "grid", "pr_check_size",
                  "queue_capacity", "timeout_ms", "split_degree", "color_order_degree",
                  "fetch_policy", "push_policy", "discrete_tail", "color_forbid_all",
                  "pr_combine"):
            setattr(c, f, int(getattr(self, f)))
        c.abort_flag = self.abort.address if self.abort is not None else None
        return c

    def key(self):
        return (self.strategy, self.worker, self.fetch, self.queue_layout, self.grid,
                self.pr_check_size, self.queue_capacity, self.color_order_degree, self.split_degree,
                self.fetch_policy, self.push_policy, self.discrete_tail, self.color_forbid_all,
                self.pr_combine)


@dataclass
class Stats:
    status: int = 0
    tasks_popped: int = 0
    tasks_pushed: int = 0
    edges_scanned: int = 0
    rounds: int = 0
    device_ms: float = 0.0
    kernel_ms: float = 0.0
    push_retries: int = 0
    idle_iterations: int = 0
    steals: int = 0
    hub_posts: int = 0
    combined_updates: int = 0
    combine_atomics: int = 0
    extra: dict = field(default_factory=dict)


class AbortFlag:
    """A word of pinned host memory that stops the runs configured with it
    (``Config(abort=flag)``) when set: the workers poll it and end the run
    with EABORTED.  Any host thread may call ``set``."""

    def __init__(self):
        p = ctypes.c_void_p()
        _check(_load().atos_host_alloc(64, ctypes.byref(p)), "atos_host_alloc")
        self._p = p
        self._word = ctypes.c_uint32.from_address(p.value)
        self._word.value = 0

    @property
    def address(self) -> int:
        return self._p.value

    def set(self):
        self._word.value = 1

    def clear(self):
        self._word.value = 0

    def close(self):
        if getattr(self, "_p", None) is not None:
            _load().atos_host_free(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def library_path() -> str:
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(
            f"libatos.so is not built ({_LIB_PATH}); build it with "
            "`python -m paper_2112_00132_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i32, i64, u32, u64, f32 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                   ctypes.c_uint32, ctypes.c_uint64, ctypes.c_float)
    cfgp, stp = ctypes.POINTER(_Config), ctypes.POINTER(_Stats)
    sig = {
        "atos_graph_load": [vp, i32, vp, i64, i64, u32, vp, ctypes.POINTER(vp)],
        "atos_graph_free": [vp],
        "atos_graph_info": [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)],
        "atos_workspace_bytes": [vp, i32, cfgp, ctypes.POINTER(ctypes.c_size_t)],
        "atos_workspace_stats": [vp, vp, stp],
        "atos_bfs": [vp, i64, vp, vp, ctypes.c_size_t, cfgp, vp, stp],
        "atos_bfs_noalloc": [vp, i64, vp, cfgp, vp, stp],
        "atos_pagerank": [vp, f32, f32, vp, vp, vp, ctypes.c_size_t, cfgp, vp, stp],
        "atos_ppr": [vp, i64, f32, f32, vp, vp, vp, ctypes.c_size_t, cfgp, vp, stp],
        "atos_server_arena_bytes": [ctypes.POINTER(vp), i32, ctypes.POINTER(_ServerConfig),
                                    ctypes.POINTER(ctypes.c_size_t)],
        "atos_server_create": [ctypes.POINTER(vp), i32, ctypes.POINTER(_ServerConfig), vp,
                               ctypes.c_size_t, ctypes.POINTER(vp)],
        "atos_server_start": [vp, vp],
        "atos_server_submit": [vp, ctypes.POINTER(_Query), ctypes.POINTER(u64)],
        "atos_server_poll": [vp, ctypes.POINTER(_Completion), i32, ctypes.POINTER(i32)],
        "atos_server_release": [vp, u64],
        "atos_server_stop": [vp, stp],
        "atos_server_destroy": [vp],
        "atos_server_snapshot": [vp, i32, ctypes.POINTER(u64), i64, ctypes.POINTER(i64)],
        "atos_host_alloc": [ctypes.c_size_t, ctypes.POINTER(vp)],
        "atos_host_free": [vp],
        "atos_trace_attach": [vp, ctypes.c_size_t],
        "atos_color": [vp, u64, vp, vp, vp, ctypes.c_size_t, cfgp, vp, stp],
        "atos_batch_plan": [vp, ctypes.POINTER(_BatchInstance), i32, f32, f32, cfgp, vp,
                            ctypes.POINTER(vp)],
        "atos_batch_free": [vp],
        "atos_batch_workspace_bytes": [vp, ctypes.POINTER(ctypes.c_size_t)],
        "atos_batch_run": [vp, vp, vp, vp, ctypes.c_size_t, vp, stp],
        "atos_batch_capture": [vp, vp, vp, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)],
        "atos_exec_launch": [vp, vp],
        "atos_exec_free": [vp],
        "atos_autotune": [vp, i32, i64, f32, f32, u64, vp, vp, vp, ctypes.c_size_t, cfgp, i32, vp,
                          ctypes.POINTER(_TuneResult), i32, ctypes.POINTER(i32), cfgp],
        "atos_batch_set_config": [vp, cfgp],
        "atos_microbench": [i32, vp, ctypes.c_size_t, i64, i32, i32, vp, ctypes.POINTER(f32)],
        "atos_batch_autotune": [vp, vp, vp, vp, ctypes.c_size_t, i32, vp,
                                ctypes.POINTER(_TuneResult), i32, ctypes.POINTER(i32), cfgp],
        "atos_tune_set_progress": [vp, vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.atos_strerror.argtypes = [ctypes.c_int]
    lib.atos_strerror.restype = ctypes.c_char_p
    lib.atos_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status: int, where: str):
    if status != 0:
        raise AtosError(status, where)


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stats_from(st: _Stats) -> Stats:
    return Stats(status=st.status, tasks_popped=st.tasks_popped, tasks_pushed=st.tasks_pushed,
                 edges_scanned=st.edges_scanned, rounds=st.rounds, device_ms=st.device_ms,
                 kernel_ms=st.kernel_ms, push_retries=st.push_retries,
                 idle_iterations=st.idle_iterations, steals=st.steals, hub_posts=st.hub_posts,
                 combined_updates=st.combined_updates, combine_atomics=st.combine_atomics)


class Graph:
    """A CSR graph resident on the current HIP device.

    ``offsets`` (int32 or int64, n+1) and ``cols`` (int32, m) are device
    tensors; the graph keeps references to them.  ``symmetric`` asserts that
    every edge is stored in both directions (required by PageRank and
    colouring)."""

    def __init__(self, offsets, cols, symmetric: bool = True, validate: bool = False,
                 stream=None):
        import torch
        lib = _load()
        if offsets.device.type != "cuda" or cols.device.type != "cuda":
            raise ValueError("offsets and cols must be device tensors")
        if offsets.dtype not in (torch.int32, torch.int64) or cols.dtype != torch.int32:
            raise ValueError("offsets must be int32/int64 and cols int32")
        self.offsets = offsets.contiguous()
        self.cols = cols.contiguous()
        self.n = int(self.offsets.numel()) - 1
        self.m = int(self.cols.numel())
        flags = (GRAPH_SYMMETRIC if symmetric else 0) | (GRAPH_VALIDATE if validate else 0)
        h = ctypes.c_void_p()
        _check(lib.atos_graph_load(_ptr(self.offsets), 1 if self.offsets.dtype == torch.int64 else 0,
                                   _ptr(self.cols), self.n, self.m, flags, _stream_handle(stream),
                                   ctypes.byref(h)), "atos_graph_load")
        self._h = h
        n, m, d = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib.atos_graph_info(h, ctypes.byref(n), ctypes.byref(m), ctypes.byref(d)),
               "atos_graph_info")
        self.max_degree = int(d.value)
        self._ws = {}

    @classmethod
    def from_csr(cls, offsets, cols, device="cuda", offsets_int64: bool = True, **kw):
        """Upload host CSR arrays (numpy or torch) to the device."""
        import torch
        o = torch.as_tensor(offsets).to(torch.int64 if offsets_int64 else torch.int32)
        c = torch.as_tensor(cols).to(torch.int32)
        return cls(o.to(device), c.to(device), **kw)

    def workspace_bytes(self, app: int, cfg: Config | None = None) -> int:
        b = ctypes.c_size_t()
        c = (cfg or Config())._c()
        _check(_load().atos_workspace_bytes(self._h, app, ctypes.byref(c), ctypes.byref(b)),
               "atos_workspace_bytes")
        return int(b.value)

    def workspace(self, app: int, cfg: Config | None = None):
        """Device workspace for ``app`` under ``cfg``, allocated once and reused."""
        import torch
        nbytes = self.workspace_bytes(app, cfg)
        key = (app, (cfg or Config()).key())
        ws = self._ws.get(key)
        if ws is None or ws.numel() < nbytes:
            ws = torch.empty(nbytes, dtype=torch.uint8, device=self.offsets.device)
            ws[:_WS_HEADER_BYTES].zero_()  # fresh memory: the library re-initialises the rest
            self._ws[key] = ws
        return ws

    def last_status(self, app: int, cfg: Config | None = None, stream=None) -> Stats:
        """Outcome and counters of the last run of ``app`` under ``cfg`` on this
        graph's cached workspace (waits for ``stream``)."""
        st = _Stats()
        ws = self.workspace(app, cfg)
        _check(_load().atos_workspace_stats(_ptr(ws), _stream_handle(stream), ctypes.byref(st)),
               "atos_workspace_stats")
        return _stats_from(st)

    def close(self):
        if getattr(self, "_h", None):
            _load().atos_graph_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


EOVERFLOW = 3


def default_queue_capacity(g: "Graph", app: int, cfg: Config | None = None) -> int:
    """Entries per worklist ring the library picks when ``queue_capacity`` is 0:
    all rings together hold 4n (BFS) or 8n (PageRank, colouring) entries, at
    least 2^16 per ring, rounded up to a power of two."""
    cfg = cfg or Config()
    nq = 1 if cfg.queue_layout == QUEUE_GLOBAL else 8
    want = max(1 << 16, (4 if app == APP_BFS else 8) * max(g.n, 1) // nq)
    return 1 << (int(want) - 1).bit_length()


def _run(fn_name, g: Graph, app: int, cfg, stream, want_stats, check, *args,
         overflow_retries: int = 2):
    """Call ``fn_name`` with the graph's cached workspace.  The device's
    outcome (ring overflow, deadline, abort) is known only once the run ends:
    with ``stats`` the call waits and returns the counters; otherwise with
    ``check`` (the default) it waits for the run and reads the workspace's
    status word; either way a device error raises AtosError.  A ring overflow
    is retried up to ``overflow_retries`` times with twice the ring capacity
    (a new workspace) before it raises.  With ``check=False`` and no stats the
    call only enqueues the run, and ``Graph.last_status`` reads the outcome
    later."""
    import dataclasses
    cfg = cfg or Config()
    lib = _load()
    for attempt in range(overflow_retries + 1):
        ws = g.workspace(app, cfg)
        c = cfg._c()
        st = _Stats()
        status = getattr(lib, fn_name)(g._h, *args, _ptr(ws), ws.numel(), ctypes.byref(c),
                                       _stream_handle(stream),
                                       ctypes.byref(st) if want_stats else None)
        _check(status, fn_name)
        if not (want_stats or check):
            return None
        if not want_stats:
            _check(lib.atos_workspace_stats(_ptr(ws), _stream_handle(stream), ctypes.byref(st)),
                   "atos_workspace_stats")
        if st.status == EOVERFLOW and attempt < overflow_retries:
            cap = cfg.queue_capacity or default_queue_capacity(g, app, cfg)
            cfg = dataclasses.replace(cfg, queue_capacity=2 * cap)
            continue
        if st.status != 0:
            raise AtosError(st.status, fn_name + " (device)")
        return _stats_from(st) if want_stats else None


def bfs(g: Graph, source: int, cfg: Config | None = None, out=None, stream=None,
        stats: bool = False, check: bool = True, overflow_retries: int = 2):
    """Hop depths from ``source`` (int32 device tensor, -1 = unreached)."""
    import torch
    depth = out if out is not None else torch.empty(g.n, dtype=torch.int32, device=g.cols.device)
    st = _run("atos_bfs", g, APP_BFS, cfg, stream, stats, check, ctypes.c_int64(int(source)),
              _ptr(depth), overflow_retries=overflow_retries)
    return (depth, st) if stats else depth


def bfs_noalloc(g: Graph, source: int, cfg: Config | None = None, out=None, stream=None,
                stats: bool = False):
    """``bfs`` on the library's fixed per-GPU scratch (atos_bfs_noalloc): the
    call allocates no device memory.  Graphs whose BFS workspace exceeds
    ``NOALLOC_SCRATCH_BYTES`` raise ENOMEM.  With ``stats`` the counters come
    back without device times."""
    import torch
    depth = out if out is not None else torch.empty(g.n, dtype=torch.int32, device=g.cols.device)
    c = (cfg or Config())._c()
    st = _Stats()
    _check(_load().atos_bfs_noalloc(g._h, ctypes.c_int64(int(source)), _ptr(depth), ctypes.byref(c),
                                    _stream_handle(stream), ctypes.byref(st) if stats else None),
           "atos_bfs_noalloc")
    if stats:
        if st.status != 0:
            raise AtosError(st.status, "atos_bfs_noalloc (device)")
        return depth, _stats_from(st)
    return depth


NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024 + 64 * 1024


def pagerank(g: Graph, damping: float = 0.85, epsilon: float = 1e-7, cfg: Config | None = None,
             out=None, residual=None, stream=None, stats: bool = False, check: bool = True,
             overflow_retries: int = 2):
    """Residual-push PageRank (FP32 ranks, unnormalised: sum ~ n)."""
    import torch
    rank = out if out is not None else torch.empty(g.n, dtype=torch.float32, device=g.cols.device)
    st = _run("atos_pagerank", g, APP_PAGERANK, cfg, stream, stats, check, ctypes.c_float(damping),
              ctypes.c_float(epsilon), _ptr(rank), _ptr(residual), overflow_retries=overflow_retries)
    return (rank, st) if stats else rank


def ppr(g: Graph, source: int, damping: float = 0.85, epsilon: float = 1e-6,
        cfg: Config | None = None, out=None, residual=None, stream=None, stats: bool = False,
        check: bool = True, overflow_retries: int = 2):
    """Personalized PageRank from ``source`` (FP32 ranks of x = (1-d) e_s + d A D^-1 x)."""
    import torch
    rank = out if out is not None else torch.empty(g.n, dtype=torch.float32, device=g.cols.device)
    st = _run("atos_ppr", g, APP_PAGERANK, cfg, stream, stats, check, ctypes.c_int64(int(source)),
              ctypes.c_float(damping), ctypes.c_float(epsilon), _ptr(rank), _ptr(residual),
              overflow_retries=overflow_retries)
    return (rank, st) if stats else rank


def color(g: Graph, seed: int = 3, cfg: Config | None = None, out=None, stream=None,
          stats: bool = False, check: bool = True, overflow_retries: int = 2):
    """Speculative greedy colouring: (colour tensor int32, colour-count device scalar)."""
    import torch
    col = out if out is not None else torch.empty(g.n, dtype=torch.int32, device=g.cols.device)
    ncol = torch.zeros(1, dtype=torch.int32, device=g.cols.device)
    st = _run("atos_color", g, APP_COLOR, cfg, stream, stats, check, ctypes.c_uint64(int(seed)),
              _ptr(col), _ptr(ncol), overflow_retries=overflow_retries)
    return (col, ncol, st) if stats else (col, ncol)


def _config_from(c: _Config) -> Config:
    return Config(strategy=c.strategy, worker=c.worker, fetch=c.fetch, queue_layout=c.queue_layout,
                  grid=c.grid, pr_check_size=c.pr_check_size, queue_capacity=c.queue_capacity,
                  timeout_ms=c.timeout_ms, split_degree=c.split_degree,
                  color_order_degree=c.color_order_degree, fetch_policy=c.fetch_policy,
                  push_policy=c.push_policy, discrete_tail=c.discrete_tail,
                  color_forbid_all=c.color_forbid_all)


_TUNE_PROGRESS = ctypes.CFUNCTYPE(None, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.POINTER(_TuneResult), ctypes.c_void_p)


class _TuneProgress:
    """Registers ``fn(done, planned, point_dict)`` as the tuner's progress
    callback for the duration of a ``with`` block."""

    def __init__(self, fn):
        self.fn = fn
        self.cb = None

    def __enter__(self):
        if self.fn is not None:
            def call(done, planned, res, _user):
                self.fn(int(done), int(planned), _tune_table(res, 1)[0])
            self.cb = _TUNE_PROGRESS(call)
            _check(_load().atos_tune_set_progress(ctypes.cast(self.cb, ctypes.c_void_p), None),
                   "atos_tune_set_progress")
        return self

    def __exit__(self, *exc):
        if self.cb is not None:
            _load().atos_tune_set_progress(None, None)
            self.cb = None


def _tune_table(res, n):
    return [{"strategy": res[i].cfg.strategy, "worker": res[i].cfg.worker, "fetch": res[i].cfg.fetch,
             "queue_layout": res[i].cfg.queue_layout, "push_policy": res[i].cfg.push_policy,
             "median_ms": float(res[i].median_ms), "status": int(res[i].status)} for i in range(n)]


def graph_class(g: "Graph") -> str:
    """'scale-free' when the largest degree dwarfs the average, else 'mesh'."""
    avg = g.m / max(g.n, 1)
    return "scale-free" if g.max_degree > 32 * max(avg, 1.0) else "mesh"


def tune_key(g: "Graph", app: int) -> str:
    import math
    return f"{app}:{graph_class(g)}:e{int(math.log2(max(g.m, 1)))}"


def autotune(g: Graph, app: int, source: int = 0, damping: float = 0.85, epsilon: float = 1e-7,
             seed: int = 3, reps: int = 3, base: Config | None = None, cache: str | None = None,
             stream=None, progress=None):
    """Sweep worker size x fetch x queue layout for ``app`` on ``g``, then the
    kernel strategies and push policies at the winning launch shape (native
    sweep in the library); returns (best Config, table).  With ``cache`` (a
    JSON path), a result stored under (app, graph class, size bucket) is
    reused and new results are added."""
    import json
    import torch
    key = tune_key(g, app)
    if cache and os.path.exists(cache):
        with open(cache) as f:
            stored = json.load(f)
        if key in stored:
            return Config(**stored[key]["config"]), stored[key]["table"]
    base = base or Config()
    dev = g.cols.device
    out = torch.empty(g.n, dtype=torch.float32 if app == APP_PAGERANK else torch.int32, device=dev)
    residual = torch.empty(g.n, dtype=torch.float32, device=dev) if app == APP_PAGERANK else None
    ws = g.workspace(app, base)
    res = (_TuneResult * 128)()
    n = ctypes.c_int32()
    best = _Config()
    c = base._c()
    with _TuneProgress(progress):
        _check(_load().atos_autotune(g._h, app, int(source), ctypes.c_float(damping),
                                     ctypes.c_float(epsilon), ctypes.c_uint64(seed), _ptr(out),
                                     _ptr(residual), _ptr(ws), ws.numel(), ctypes.byref(c), int(reps),
                                     _stream_handle(stream), res, 128, ctypes.byref(n),
                                     ctypes.byref(best)), "atos_autotune")
    cfg = _config_from(best)
    table = _tune_table(res, n.value)
    if cache:
        stored = {}
        if os.path.exists(cache):
            with open(cache) as f:
                stored = json.load(f)
        stored[key] = {"config": vars(cfg), "table": table}
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        with open(cache, "w") as f:
            json.dump(stored, f, indent=1)
    return cfg, table


MB_KINDS = {"copy": 0, "atomic_add_f32": 1, "atomic_min_u32": 2, "same_address": 3,
            "fences": 4, "gather_plain": 5, "gather_coherent": 6, "litmus_mp": 7,
            "atomic_add_f64": 8, "clock": 9, "atomic_add_f64_noret": 10, "atomic_add_f64_xcd": 11}


def microbench(kind: str, buf, iters: int = 0, grid: int = 0, block: int = 256, stream=None) -> float:
    """Run one primitive microbenchmark on device buffer ``buf``; returns ms."""
    import torch
    if grid == 0:
        grid = torch.cuda.get_device_properties(buf.device).multi_processor_count * 8
    ms = ctypes.c_float()
    _check(_load().atos_microbench(MB_KINDS[kind], _ptr(buf), buf.numel() * buf.element_size(),
                                   int(iters), int(grid), int(block), _stream_handle(stream),
                                   ctypes.byref(ms)), "atos_microbench")
    return float(ms.value)


TRACE_DTYPE = [("t_begin", "<u8"), ("t_end", "<u8"), ("worker", "<u4"), ("tasks", "<u4"),
               ("edges", "<u4"), ("vertex", "<u4")]
TRACE_HUB_CHUNK = 0x80000000
TRACE_BSP_LEVEL = 0x40000000


class Trace:
    """Per-batch event trace of the persistent worker kernel (atos_trace_attach):
    while attached, every persistent launch on the buffer's device appends one
    record per batch a worker processes.  Use as a context manager, or call
    attach()/detach(); records() returns the stored records as a numpy
    structured array (fields of TRACE_DTYPE) once the traced work is done."""

    def __init__(self, records: int = 1 << 20, device="cuda"):
        import torch
        self.buf = torch.zeros(64 + 32 * int(records), dtype=torch.uint8, device=device)

    def attach(self):
        _check(_load().atos_trace_attach(_ptr(self.buf), self.buf.numel()), "atos_trace_attach")
        return self

    def detach(self):
        _check(_load().atos_trace_attach(None, 0), "atos_trace_attach")

    def __enter__(self):
        return self.attach()

    def __exit__(self, *exc):
        self.detach()

    def count(self) -> int:
        """Records appended since attach (may exceed the capacity)."""
        return int(self.buf[:8].view(__import__("torch").int64).item())

    def clock_khz(self) -> int:
        """Rate of the records' t_begin / t_end clock."""
        return int(self.buf[16:24].view(__import__("torch").int64).item())

    def timeline(self, bins: int = 40, useful_edges: int | None = None) -> dict:
        """Throughput over time from the worker-batch records: per time bin,
        edges scanned per second (each batch's edges spread evenly over its
        duration) and the mean number of busy workers.  With ``useful_edges``
        (the edges the work needs, e.g. a level-synchronous run's count) each
        bin's throughput is also reported normalised by the run's overwork,
        i.e. multiplied by useful_edges / edges scanned (the paper's normalised
        throughput, section 6.4)."""
        import numpy as np
        r = self.records()
        r = r[(r["tasks"] & TRACE_BSP_LEVEL) == 0]
        if r.size == 0:
            return {"ms": [], "gteps": [], "busy_workers": []}
        tick_ms = 1.0 / self.clock_khz()
        tb = r["t_begin"].astype(np.float64)
        te = np.maximum(r["t_end"].astype(np.float64), tb + 1.0)
        t0, t1 = tb.min(), te.max()
        edges = r["edges"].astype(np.float64)
        edges_bin = np.zeros(bins)
        busy = np.zeros(bins)
        width = (t1 - t0) / bins
        for i in range(bins):
            a, b = t0 + i * width, t0 + (i + 1) * width
            ov = np.clip(np.minimum(te, b) - np.maximum(tb, a), 0.0, None)
            edges_bin[i] = (edges * ov / (te - tb)).sum()
            busy[i] = ov.sum() / width
        ms = width * tick_ms
        out = {"ms": [round((i + 0.5) * ms, 4) for i in range(bins)],
               "gteps": [round(e / (ms * 1e-3) / 1e9, 3) for e in edges_bin],
               "busy_workers": [round(b, 2) for b in busy],
               "batches": int(r.size), "span_ms": (t1 - t0) * tick_ms,
               "edges": int(edges.sum())}
        if useful_edges is not None:
            scale = useful_edges / max(edges.sum(), 1.0)
            out["overwork"] = float(edges.sum() / max(useful_edges, 1))
            out["gteps_normalised"] = [round(e * scale / (ms * 1e-3) / 1e9, 3) for e in edges_bin]
        return out

    def levels(self) -> dict:
        """Per level of the level-synchronous runs recorded (records with
        TRACE_BSP_LEVEL): level, frontier size, edges scanned and duration in
        microseconds (from the level's record to the next)."""
        import numpy as np
        r = self.records()
        r = r[(r["tasks"] & TRACE_BSP_LEVEL) != 0]
        if r.size < 2:
            return {"level": [], "frontier": [], "edges": [], "us": []}
        tick_us = 1e3 / self.clock_khz()
        t = r["t_begin"].astype(np.float64)
        e = r["edges"].astype(np.int64)
        keep = np.flatnonzero(r["worker"][1:] == r["worker"][:-1] + 1)  # consecutive levels of one run
        return {"level": r["worker"][keep].astype(int).tolist(),
                "frontier": (r["tasks"][keep] & (TRACE_BSP_LEVEL - 1)).astype(int).tolist(),
                "edges": ((e[keep + 1] - e[keep]) % (1 << 32)).astype(int).tolist(),
                "us": np.round((t[keep + 1] - t[keep]) * tick_us, 2).tolist()}

    def records(self):
        import numpy as np
        n = min(self.count(), (self.buf.numel() - 64) // 32)
        raw = self.buf[64:64 + 32 * n].cpu().numpy()
        return raw.view(np.dtype(TRACE_DTYPE))


def version() -> str:
    return _load().atos_version().decode()


class Batch:
    """Many BFS / PageRank instances over one union graph in one persistent launch.

    ``instances`` is a list of ``(app, vertex_begin, vertex_end, source)``
    tuples (app = APP_BFS or APP_PAGERANK; source ignored for PageRank),
    sorted and disjoint; each instance's edges must stay inside its range."""

    def __init__(self, g: Graph, instances, damping: float = 0.85, epsilon: float = 1e-7,
                 cfg: Config | None = None, stream=None):
        lib = _load()
        arr = (_BatchInstance * len(instances))()
        for i, (app, vb, ve, src) in enumerate(instances):
            arr[i].app, arr[i].reserved = int(app), 0
            arr[i].vertex_begin, arr[i].vertex_end, arr[i].source = int(vb), int(ve), int(src)
        self.g = g
        self.instances = list(instances)
        c = (cfg or Config())._c()
        h = ctypes.c_void_p()
        _check(lib.atos_batch_plan(g._h, arr, len(instances), ctypes.c_float(damping),
                                   ctypes.c_float(epsilon), ctypes.byref(c), _stream_handle(stream),
                                   ctypes.byref(h)), "atos_batch_plan")
        self._h = h
        b = ctypes.c_size_t()
        _check(lib.atos_batch_workspace_bytes(h, ctypes.byref(b)), "atos_batch_workspace_bytes")
        import torch
        self.ws = torch.empty(int(b.value), dtype=torch.uint8, device=g.cols.device)
        self.ws[:_WS_HEADER_BYTES].zero_()

    def run(self, state=None, residual=None, stream=None, stats: bool = False,
            check: bool = True):
        """Returns the int32 state tensor (BFS depth, or PageRank rank bits:
        use ``state.view(torch.float32)`` on PageRank ranges).  A device error
        raises AtosError unless ``check=False`` (then the call only enqueues the
        run; ``last_stats`` reads its outcome)."""
        import torch
        if state is None:
            state = torch.zeros(self.g.n, dtype=torch.int32, device=self.g.cols.device)
        st = _Stats()
        _check(_load().atos_batch_run(self._h, _ptr(state), _ptr(residual), _ptr(self.ws),
                                      self.ws.numel(), _stream_handle(stream),
                                      ctypes.byref(st) if stats else None), "atos_batch_run")
        if not stats and check:
            _check(_load().atos_workspace_stats(_ptr(self.ws), _stream_handle(stream),
                                                ctypes.byref(st)), "atos_workspace_stats")
        if (stats or check) and st.status != 0:
            raise AtosError(st.status, "atos_batch_run (device)")
        return (state, _stats_from(st)) if stats else state

    def capture(self, state, residual=None, stream=None) -> "Exec":
        """Capture one run into a hipGraph (``stream`` must not be the null stream)."""
        h = ctypes.c_void_p()
        _check(_load().atos_batch_capture(self._h, _ptr(state), _ptr(residual), _ptr(self.ws),
                                          self.ws.numel(), _stream_handle(stream),
                                          ctypes.byref(h)), "atos_batch_capture")
        return Exec(h, keep=(state, residual, self))

    def set_config(self, cfg: Config):
        c = cfg._c()
        _check(_load().atos_batch_set_config(self._h, ctypes.byref(c)), "atos_batch_set_config")

    def tune_key(self) -> str:
        """Cache key of this batch: its union graph's class and size bucket."""
        return "batch:" + tune_key(self.g, 0).split(":", 1)[1]

    def autotune(self, reps: int = 3, stream=None, cache: str | None = None, progress=None):
        """Native sweep of worker size x fetch x layout for this batch, then
        both push policies at the winning shape; the batch keeps its
        configuration.  Returns (best Config, table).  With ``cache`` (a JSON
        path) a result stored under ``tune_key()`` is reused, and a new one is
        stored."""
        import json
        import torch
        key = self.tune_key()
        if cache and os.path.exists(cache):
            with open(cache) as f:
                stored = json.load(f)
            if key in stored:
                return Config(**stored[key]["config"]), stored[key]["table"]
        state = torch.zeros(self.g.n, dtype=torch.int32, device=self.g.cols.device)
        res = (_TuneResult * 128)()
        n = ctypes.c_int32()
        best = _Config()
        with _TuneProgress(progress):
            _check(_load().atos_batch_autotune(self._h, _ptr(state), None, _ptr(self.ws),
                                               self.ws.numel(), int(reps), _stream_handle(stream),
                                               res, 128, ctypes.byref(n), ctypes.byref(best)),
                   "atos_batch_autotune")
        cfg, table = _config_from(best), _tune_table(res, n.value)
        if cache:
            stored = {}
            if os.path.exists(cache):
                with open(cache) as f:
                    stored = json.load(f)
            stored[key] = {"config": vars(cfg), "table": table}
            with open(cache, "w") as f:
                json.dump(stored, f, indent=1)
        return cfg, table

    def last_stats(self, stream=None) -> Stats:
        st = _Stats()
        _check(_load().atos_workspace_stats(_ptr(self.ws), _stream_handle(stream), ctypes.byref(st)),
               "atos_workspace_stats")
        return _stats_from(st)

    def close(self):
        if getattr(self, "_h", None):
            _load().atos_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Exec:
    """An instantiated hipGraph of one batch run."""

    def __init__(self, h, keep):
        self._h = h
        self._keep = keep

    def launch(self, stream=None):
        _check(_load().atos_exec_launch(self._h, _stream_handle(stream)), "atos_exec_launch")

    def close(self):
        if getattr(self, "_h", None):
            _load().atos_exec_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class ServerConfig:
    """Daemon configuration (mirrors ``atos_server_config``; 0 = library default)."""
    worker: int = 0
    fetch: int = 0
    grid: int = 0
    max_queries: int = 0
    queue_capacity: int = 0
    timeout_ms: int = 0
    queue_layout: int = QUEUE_AUTO  # a ring per XCD (AUTO), or QUEUE_GLOBAL (one shared ring)
    push_policy: int = 0  # with per-XCD rings: PUSH_QUERY (AUTO), PUSH_OWN or PUSH_SHALLOWEST

    def _c(self) -> _ServerConfig:
        c = _ServerConfig()
        for f in ("worker", "fetch", "grid", "max_queries", "queue_capacity", "timeout_ms",
                  "queue_layout", "push_policy"):
            setattr(c, f, int(getattr(self, f)))
        return c


@dataclass
class Completion:
    query_id: int
    tag: int
    status: int
    app: int
    graph: int
    state_offset: int
    tasks: int
    edges: int
    device_us: float


def server_arena_bytes(graphs, cfg: ServerConfig | None = None) -> int:
    """Arena bytes a server over ``graphs`` needs before its state heap."""
    arr = (ctypes.c_void_p * len(graphs))(*[g._h for g in graphs])
    c = (cfg or ServerConfig())._c()
    b = ctypes.c_size_t()
    _check(_load().atos_server_arena_bytes(arr, len(graphs), ctypes.byref(c), ctypes.byref(b)),
           "atos_server_arena_bytes")
    return int(b.value)


class Server:
    """Resident query daemon over a fixed list of graphs (continuous batching).

    The daemon kernel runs on its own stream from ``start()`` until
    ``stop()``; while it runs, nothing may synchronise the whole device
    (``torch.cuda.synchronize``) or free device memory, since that would wait
    for the daemon.  With ``host_results`` the server keeps one pinned host
    block per query slot (max_queries blocks of 8 bytes per vertex of the
    largest graph); the daemon writes every result there before it posts the
    completion, so ``result`` needs no GPU call.  Without it results stay in
    the device arena (``Completion.state_offset``) until release."""

    def __init__(self, graphs, arena_bytes: int | None = None, cfg: ServerConfig | None = None,
                 heap_fraction: float = 0.5, host_results: bool = True):
        import torch
        lib = _load()
        self.graphs = list(graphs)
        self._arr = (ctypes.c_void_p * len(self.graphs))(*[g._h for g in self.graphs])
        self._cfg = (cfg or ServerConfig())._c()
        fixed = server_arena_bytes(self.graphs, cfg)
        dev = self.graphs[0].cols.device
        if arena_bytes is None:
            free, _ = torch.cuda.mem_get_info(dev)
            arena_bytes = fixed + int(max(free - fixed, 0) * heap_fraction)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=dev)
        h = ctypes.c_void_p()
        _check(lib.atos_server_create(self._arr, len(self.graphs), ctypes.byref(self._cfg),
                                      _ptr(self.arena), self.arena.numel(), ctypes.byref(h)),
               "atos_server_create")
        self._h = h
        self.stream = torch.cuda.Stream(device=dev)
        self.running = False
        self._host = None
        self._blocks, self._free_blocks, self._block_of = [], [], {}
        if host_results:
            slots = self._cfg.max_queries or 256
            self._block_bytes = 8 * max(g.n for g in self.graphs)  # PageRank: rank + residue
            p = ctypes.c_void_p()
            _check(lib.atos_host_alloc(slots * self._block_bytes, ctypes.byref(p)), "atos_host_alloc")
            self._host = p
            self._free_blocks = list(range(slots))[::-1]

    def start(self):
        _check(_load().atos_server_start(self._h, ctypes.c_void_p(self.stream.cuda_stream)),
               "atos_server_start")
        self.running = True

    def submit(self, graph: int, app: int, source: int, damping: float = 0.85,
               epsilon: float = 1e-6, tag: int = 0):
        """Query id, or None when the server has no room right now (EAGAIN)."""
        out = None
        block = None
        if self._host is not None:
            if not self._free_blocks:
                return None
            block = self._free_blocks.pop()
            out = self._host.value + block * self._block_bytes
        q = _Query(graph=int(graph), app=int(app), source=int(source), damping=float(damping),
                   epsilon=float(epsilon), tag=int(tag), out=out)
        qid = ctypes.c_uint64()
        st = _load().atos_server_submit(self._h, ctypes.byref(q), ctypes.byref(qid))
        if st != 0 and block is not None:
            self._free_blocks.append(block)
        if st == EAGAIN:
            return None
        _check(st, "atos_server_submit")
        if block is not None:
            self._block_of[int(qid.value)] = block
        return int(qid.value)

    def poll(self, max_n: int = 256):
        buf = (_Completion * max_n)()
        n = ctypes.c_int32()
        _check(_load().atos_server_poll(self._h, buf, max_n, ctypes.byref(n)), "atos_server_poll")
        return [Completion(c.query_id, c.tag, c.status, c.app, c.graph, c.state_offset, c.tasks,
                           c.edges, c.device_us) for c in buf[:n.value]]

    def result(self, c: Completion):
        """Copy of a completed query's result (from the pinned block the daemon
        wrote): int64 depths (-1 = unreached) for BFS, (FP32 rank, FP32
        residue) for PageRank."""
        import numpy as np
        if self._host is None:
            raise RuntimeError("server created without host_results")
        n = self.graphs[c.graph].n
        addr = self._host.value + self._block_of[c.query_id] * self._block_bytes
        if c.app == APP_BFS:
            a = np.ctypeslib.as_array((ctypes.c_int32 * n).from_address(addr)).copy()
            return a.astype(np.int64)
        a = np.ctypeslib.as_array((ctypes.c_float * (2 * n)).from_address(addr)).copy()
        return a[:n], a[n:]

    def release(self, query_id: int):
        _check(_load().atos_server_release(self._h, int(query_id)), "atos_server_release")
        block = self._block_of.pop(int(query_id), None)
        if block is not None:
            self._free_blocks.append(block)

    def snapshot(self, ring_words: int = 8) -> dict:
        """The daemon's counters, busy slots and the first ring words at every
        ring's head, decoded (taken by a worker of the running daemon)."""
        cap = 15 + 3 * 8 + 4 * 2048 + ring_words * 8
        buf = (ctypes.c_uint64 * cap)()
        n = ctypes.c_int64()
        _check(_load().atos_server_snapshot(self._h, int(ring_words), buf, cap, ctypes.byref(n)),
               "atos_server_snapshot")
        w = list(buf[:n.value])
        nq, capacity, nslots = w[6], w[7], w[8]
        out = {"status": w[0], "submit_head": w[1], "comp_tail": w[2], "active": w[3],
               "admitted": w[4], "completed": w[5], "rings": [], "slots": {},
               "timeout_after_s": (w[10] - w[9]) / (w[11] * 1e3) if w[10] else None,
               "epoch": w[12], "epoch_started": w[13], "epoch_timed_out": w[14]}
        i = 15
        for q in range(nq):
            out["rings"].append({"head": w[i], "tail": w[i + 1], "done": w[i + 2]})
            i += 3
        for sl in range(nslots):
            qid, pending, init_left, ag = w[i:i + 4]
            if pending:
                out["slots"][sl] = {"query_id": qid, "pending": pending, "init_left": init_left,
                                    "app": ag >> 32, "graph": ag & 0xFFFFFFFF}
            i += 4
        lap_bits = int(capacity).bit_length() - 1
        for q in range(nq):
            words = []
            for j in range(ring_words):
                x = w[i]
                i += 1
                pos = out["rings"][q]["head"] + j
                tag = x >> 48
                full = tag == ((2 * (pos >> lap_bits) + 1) & 0xFFFF)
                words.append({"pos": pos, "tag": tag, "full": bool(full), "slot": (x >> 37) & 0x7FF,
                              "kind": (x >> 35) & 3, "vertex": (x >> 10) & 0x1FFFFFF})
            out["rings"][q]["words"] = words
        return out

    def stop(self) -> Stats:
        st = _Stats()
        status = _load().atos_server_stop(self._h, ctypes.byref(st))
        self.running = False
        _check(status, "atos_server_stop")
        return _stats_from(st)

    def close(self):
        if getattr(self, "_h", None):
            _load().atos_server_destroy(self._h)
            self._h = None
            self.running = False
        if getattr(self, "_host", None) is not None:
            _load().atos_host_free(self._host)  # after the daemon has stopped
            self._host = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
