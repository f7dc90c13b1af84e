"""Result checkers used by the tests (test infrastructure, numpy only).

Each checker returns a list of human-readable violations (empty = pass), so
a test can report what went wrong.  They characterise a correct result by
properties that hold for every correct answer and can be evaluated at any
graph size without trusting an implementation.
"""
from __future__ import annotations

import numpy as np


def _edges(g):
    deg = np.diff(np.asarray(g.offsets, dtype=np.int64))
    src = np.repeat(np.arange(g.n, dtype=np.int64), deg)
    return src, np.asarray(g.cols, dtype=np.int64), deg


def bfs_certificate(g, source: int, depth: np.ndarray, limit: int = 10) -> list[str]:
    """BFS depths are exactly the hop distances iff
    (1) d(source) = 0 and every other reached vertex has d >= 1;
    (2) every edge with both ends reached has |d(u) - d(v)| <= 1;
    (3) no edge joins a reached and an unreached vertex (unreached = -1);
    (4) every reached v != source has a neighbour u with d(u) = d(v) - 1.
    (1)+(2) give d <= dist, (4) gives d >= dist by induction."""
    d = np.asarray(depth).astype(np.int64)
    out: list[str] = []
    if d.shape != (g.n,):
        return [f"depth has shape {d.shape}, expected ({g.n},)"]
    if g.n == 0:
        return out
    if d[source] != 0:
        out.append(f"d(source={source}) = {d[source]}")
    bad = np.flatnonzero((d == 0) & (np.arange(g.n) != source))
    if bad.size:
        out.append(f"{bad.size} non-source vertices at depth 0, e.g. {bad[:limit].tolist()}")
    if (d < -1).any():
        out.append("depth below -1")
    src, dst, _ = _edges(g)
    ru, rv = d[src] >= 0, d[dst] >= 0
    both = ru & rv
    gap = np.abs(d[src] - d[dst]) > 1
    e = np.flatnonzero(both & gap)
    if e.size:
        out.append(f"{e.size} edges with |d(u)-d(v)| > 1, e.g. "
                   f"{[(int(src[i]), int(dst[i]), int(d[src[i]]), int(d[dst[i]])) for i in e[:limit]]}")
    e = np.flatnonzero(ru != rv)
    if e.size:
        out.append(f"{e.size} edges between reached and unreached, e.g. "
                   f"{[(int(src[i]), int(dst[i])) for i in e[:limit]]}")
    has_parent = np.zeros(g.n, dtype=bool)
    par = both & (d[dst] == d[src] - 1)
    has_parent[src[par]] = True
    need = (d > 0) & ~has_parent
    bad = np.flatnonzero(need)
    if bad.size:
        out.append(f"{bad.size} reached vertices without a parent, e.g. {bad[:limit].tolist()}")
    return out


def coloring_violations(g, color: np.ndarray, limit: int = 10) -> list[str]:
    """A proper colouring: every colour >= 0 and no edge u-v with c(u) = c(v).
    First-fit also guarantees c(v) <= deg(v) (at most deg(v) colours can be
    forbidden when v picks), which every schedule of the speculative method
    preserves because each assignment is a first-fit choice."""
    c = np.asarray(color).astype(np.int64)
    out: list[str] = []
    if c.shape != (g.n,):
        return [f"colour array has shape {c.shape}, expected ({g.n},)"]
    neg = np.flatnonzero(c < 0)
    if neg.size:
        out.append(f"{neg.size} uncoloured vertices, e.g. {neg[:limit].tolist()}")
    src, dst, deg = _edges(g)
    e = np.flatnonzero(c[src] == c[dst])
    if e.size:
        out.append(f"{e.size // 2} monochromatic edges, e.g. "
                   f"{[(int(src[i]), int(dst[i]), int(c[src[i]])) for i in e[:limit]]}")
    big = np.flatnonzero(c > deg)
    if big.size:
        out.append(f"{big.size} vertices with colour > degree, e.g. {big[:limit].tolist()}")
    return out


def pagerank_violations(g, rank: np.ndarray, x_ref: np.ndarray, damping: float, epsilon: float,
                        rel_tol: float | None = 1e-5, ref_bound: np.ndarray | None = None,
                        slack_ulps: float = 64.0, limit: int = 10) -> list[str]:
    """Accuracy of a push-residual PageRank against the FP64 fixed point.

    (a) |p(v) - x(v)| <= rel_tol * max(1, x(v))           (tolerance; skipped
        when rel_tol is None)
    (b) -slack <= x(v) - p(v) <= deg(v)*eps/(1-d) + slack  (one-sided bound:
        the push method leaves residue r <= eps, and x - p = (I - d A D^-1)^-1 r
        with (A D^-1)^k = D P^k D^-1, P row-stochastic).
    slack covers the oracle's own error bound plus FP32 rounding of p
    (``slack_ulps`` FP32 ulps of x(v))."""
    p = np.asarray(rank, dtype=np.float64)
    x = np.asarray(x_ref, dtype=np.float64)
    out: list[str] = []
    if p.shape != (g.n,):
        return [f"rank has shape {p.shape}, expected ({g.n},)"]
    if not np.isfinite(p).all():
        out.append("non-finite rank values")
        return out
    err = np.abs(p - x)
    tol = (rel_tol if rel_tol is not None else np.inf) * np.maximum(1.0, x)
    bad = np.flatnonzero(err > tol)
    if bad.size:
        i = bad[np.argmax(err[bad] / tol[bad])]
        out.append(f"{bad.size} vertices beyond {rel_tol:g}*max(1,x); worst v={int(i)} "
                   f"p={p[i]!r} x={x[i]!r}")
    deg = np.diff(np.asarray(g.offsets, dtype=np.int64)).astype(np.float64)
    slack = slack_ulps * np.spacing(np.float32(1.0)).astype(np.float64) * np.maximum(1.0, x)
    if ref_bound is not None:
        slack = slack + ref_bound
    upper = deg * epsilon / (1.0 - damping) + slack
    gap = x - p
    bad = np.flatnonzero((gap > upper) | (gap < -slack))
    if bad.size:
        out.append(f"{bad.size} vertices outside the one-sided bound, e.g. "
                   f"{[(int(i), float(p[i]), float(x[i])) for i in bad[:limit]]}")
    return out


def pagerank_mass(g, rank: np.ndarray, residue: np.ndarray | None, damping: float) -> tuple[float, float]:
    """(observed, expected) total of rank + residue/(1-d).

    Summing x = p + (I - d A D^-1)^-1 r over all vertices: A D^-1 preserves
    the total over non-isolated vertices, so 1^T (I - d A D^-1)^-1 r =
    sum(r)/(1-d) and 1^T x = N_nonisolated + (1-d) N_isolated."""
    deg = np.diff(np.asarray(g.offsets, dtype=np.int64))
    expected = float((deg > 0).sum()) + (1.0 - damping) * float((deg == 0).sum())
    obs = float(np.sum(np.asarray(rank, dtype=np.float64)))
    if residue is not None:
        obs += float(np.sum(np.asarray(residue, dtype=np.float64))) / (1.0 - damping)
    return obs, expected


def ppr_mass(g, source: int, rank: np.ndarray, residue: np.ndarray, damping: float) -> tuple[float, float]:
    """(observed, expected) total of rank + residue/(1-d) for personalized
    PageRank from `source`: 1^T x = (1-d) 1^T (I - d A D^-1)^-1 e_s, and
    1^T A D^-1 = 1^T on non-isolated columns, so the total is 1 when the source
    has a neighbour and 1-d when it is isolated (x = (1-d) e_s)."""
    deg = np.diff(np.asarray(g.offsets, dtype=np.int64))
    expected = 1.0 if deg[source] > 0 else 1.0 - damping
    obs = float(np.sum(np.asarray(rank, dtype=np.float64)))
    obs += float(np.sum(np.asarray(residue, dtype=np.float64))) / (1.0 - damping)
    return obs, expected


def coloring_rank_violations(g, color: np.ndarray, key: np.ndarray, limit: int = 10) -> list[str]:
    """A vertex forbids only the colours of neighbours that outrank it (rank =
    (key, id)), so its colour can never exceed the number of such neighbours."""
    c = np.asarray(color).astype(np.int64)
    k = np.asarray(key).astype(np.int64)
    src, dst, _ = _edges(g)
    outr = (k[dst] > k[src]) | ((k[dst] == k[src]) & (dst > src))
    n_out = np.bincount(src[outr], minlength=g.n)
    bad = np.flatnonzero(c > n_out)
    if bad.size:
        return [f"{bad.size} vertices coloured above their count of outranking neighbours, "
                f"e.g. {[(int(v), int(c[v]), int(n_out[v])) for v in bad[:limit]]}"]
    return []
