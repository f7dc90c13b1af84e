"""Seeded synthetic graph inputs.

This module only builds inputs: undirected CSR graphs (R-MAT, perturbed
grids, small closed-form families) and source-vertex choices.  It holds none
of the graph algorithms (no traversal, ranking or colouring), so both the
GPU path and the CPU oracle can be fed from it without sharing any of the
method's arithmetic.

The paper's datasets (SuiteSparse scale-free and road graphs, Table 2) are
not available; R-MAT graphs stand in for the scale-free ones (power-law
degrees, small diameter) and grids with deleted edges and a few diagonal
shortcuts stand in for the road networks (degree <= 8, diameter in the
thousands).

CSR convention used everywhere: ``offsets`` is int64 of length n+1,
``cols`` is int32 of length offsets[-1]; every undirected edge {u, v}
appears as both u->v and v->u, neighbour lists are sorted ascending, there
are no self-loops and no duplicate edges.
"""
from __future__ import annotations

import dataclasses

import numpy as np

__all__ = [
    "CSRGraph", "csr_from_edges", "rmat_graph", "grid_graph", "largest_component",
    "permute_graph", "path_graph", "cycle_graph", "star_graph", "complete_graph",
    "full_grid_graph", "torus_graph", "random_graph", "empty_graph",
    "max_degree_vertex", "random_source", "random_nonisolated_sources",
]


@dataclasses.dataclass
class CSRGraph:
    n: int
    offsets: np.ndarray  # int64 [n+1]
    cols: np.ndarray     # int32 [m]
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.offsets[-1])

    @property
    def degrees(self) -> np.ndarray:
        return np.diff(self.offsets)

    def edge_list(self):
        """(src, dst) int64 arrays of every directed CSR entry."""
        src = np.repeat(np.arange(self.n, dtype=np.int64), self.degrees)
        return src, self.cols.astype(np.int64)


def csr_from_edges(n: int, src: np.ndarray, dst: np.ndarray, name: str = "") -> CSRGraph:
    """Symmetrize, drop self-loops and duplicates, and build a sorted CSR."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    keep = src != dst
    src, dst = src[keep], dst[keep]
    key = np.concatenate([src * n + dst, dst * n + src])
    del src, dst, keep
    key = np.unique(key)  # sorted, deduplicated
    s = key // n
    cols = (key - s * n).astype(np.int32)
    del key
    counts = np.bincount(s, minlength=n)
    del s
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    return CSRGraph(n, offsets, cols, name)


# ---------------------------------------------------------------- R-MAT
def _rmat_draw(scale: int, edge_factor: int, a: float, b: float, c: float, rng):
    """Kronecker/R-MAT edge draws: at every level pick one of four quadrants
    with probabilities a, b, c, d = 1-a-b-c and set that level's row and
    column bits."""
    m = int(edge_factor) << int(scale)
    src = np.zeros(m, dtype=np.int64)
    dst = np.zeros(m, dtype=np.int64)
    ab, abc = a + b, a + b + c
    for level in range(scale):
        u = rng.random(m)
        row = u >= ab
        col = ((u >= a) & (u < ab)) | (u >= abc)
        src |= row.astype(np.int64) << level
        dst |= col.astype(np.int64) << level
        del u, row, col
    return src, dst


def rmat_graph(scale: int, edge_factor: int, seed: int = 1, a: float = 0.57,
               b: float = 0.19, c: float = 0.19, permute_seed: int | None = None) -> CSRGraph:
    """Undirected R-MAT graph with 2**scale vertices (isolated ones kept).

    ``permute_seed`` relabels vertex IDs by a uniform random permutation drawn
    from ``default_rng(permute_seed)`` (vertex v becomes perm[v])."""
    n = 1 << scale
    rng = np.random.default_rng(seed)
    src, dst = _rmat_draw(scale, edge_factor, a, b, c, rng)
    name = f"rmat{scale}_ef{edge_factor}_s{seed}"
    if permute_seed is not None:
        perm = np.random.default_rng(permute_seed).permutation(n).astype(np.int64)
        src = perm[src]
        dst = perm[dst]
        name += f"_perm{permute_seed}"
    return csr_from_edges(n, src, dst, name)


# ---------------------------------------------------------------- grids
def largest_component(g: CSRGraph) -> CSRGraph:
    """Keep the largest connected component, relabelled in increasing
    original-ID order (so row-major grids stay row-major)."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components

    if g.n == 0:
        return g
    mat = sp.csr_matrix((np.ones(g.m, dtype=np.int8), g.cols, g.offsets), shape=(g.n, g.n))
    ncomp, labels = connected_components(mat, directed=False)
    if ncomp == 1:
        return g
    big = np.argmax(np.bincount(labels))
    keep = labels == big
    new_id = np.cumsum(keep) - 1
    src, dst = g.edge_list()
    sel = keep[src]
    return csr_from_edges(int(keep.sum()), new_id[src[sel]], new_id[dst[sel]], g.name + "_lcc")


def grid_graph(side: int, delete_frac: float = 0.2, diag_frac: float = 0.01, seed: int = 1,
               lcc: bool = True) -> CSRGraph:
    """Road-like graph: side x side 4-neighbour grid, a uniform random
    ``delete_frac`` of its edges removed, ``round(diag_frac*side**2)``
    shortcuts from a uniform vertex to a uniform diagonal neighbour (dropped
    when off-grid), then the largest component, row-major IDs."""
    rng = np.random.default_rng(seed)
    n = side * side
    ii, jj = np.meshgrid(np.arange(side, dtype=np.int64), np.arange(side, dtype=np.int64),
                         indexing="ij")
    hmask = jj < side - 1
    vmask = ii < side - 1
    hu = (ii * side + jj)[hmask]
    vu = (ii * side + jj)[vmask]
    src = np.concatenate([hu, vu])
    dst = np.concatenate([hu + 1, vu + side])
    del ii, jj, hmask, vmask, hu, vu
    m = src.size
    ndel = int(round(delete_frac * m))
    if ndel:
        keep = rng.permutation(m)[ndel:]
        keep.sort()
        src, dst = src[keep], dst[keep]
    ndiag = int(round(diag_frac * n))
    if ndiag:
        start = rng.integers(0, n, ndiag)
        direction = rng.integers(0, 4, ndiag)
        di = np.where(direction < 2, -1, 1)
        dj = np.where(direction % 2 == 0, -1, 1)
        si, sj = start // side, start % side
        ti, tj = si + di, sj + dj
        ok = (ti >= 0) & (ti < side) & (tj >= 0) & (tj < side)
        src = np.concatenate([src, start[ok]])
        dst = np.concatenate([dst, (ti * side + tj)[ok]])
    g = csr_from_edges(n, src, dst, f"grid{side}_del{delete_frac:g}_diag{diag_frac:g}_s{seed}")
    return largest_component(g) if lcc else g


def permute_graph(g: CSRGraph, perm: np.ndarray) -> CSRGraph:
    """Relabel vertex v as perm[v]."""
    perm = np.asarray(perm, dtype=np.int64)
    src, dst = g.edge_list()
    return csr_from_edges(g.n, perm[src], perm[dst], g.name + "_perm")


# ---------------------------------------------------------------- small families
def empty_graph(n: int) -> CSRGraph:
    return CSRGraph(n, np.zeros(n + 1, dtype=np.int64), np.zeros(0, dtype=np.int32), f"empty{n}")


def path_graph(n: int) -> CSRGraph:
    v = np.arange(n - 1, dtype=np.int64)
    return csr_from_edges(n, v, v + 1, f"path{n}")


def cycle_graph(n: int) -> CSRGraph:
    v = np.arange(n, dtype=np.int64)
    return csr_from_edges(n, v, (v + 1) % n, f"cycle{n}")


def star_graph(leaves: int) -> CSRGraph:
    """Centre 0 joined to leaves 1..k."""
    v = np.arange(1, leaves + 1, dtype=np.int64)
    return csr_from_edges(leaves + 1, np.zeros_like(v), v, f"star{leaves}")


def complete_graph(n: int) -> CSRGraph:
    u, v = np.triu_indices(n, 1)
    return csr_from_edges(n, u, v, f"complete{n}")


def full_grid_graph(rows: int, cols: int) -> CSRGraph:
    """Intact rows x cols 4-neighbour grid, vertex (i, j) = i*cols + j."""
    ii, jj = np.meshgrid(np.arange(rows, dtype=np.int64), np.arange(cols, dtype=np.int64),
                         indexing="ij")
    vid = ii * cols + jj
    h = jj < cols - 1
    vv = ii < rows - 1
    src = np.concatenate([vid[h], vid[vv]])
    dst = np.concatenate([vid[h] + 1, vid[vv] + cols])
    return csr_from_edges(rows * cols, src, dst, f"fullgrid{rows}x{cols}")


def torus_graph(rows: int, cols: int) -> CSRGraph:
    """rows x cols torus (4-regular when rows, cols >= 3)."""
    ii, jj = np.meshgrid(np.arange(rows, dtype=np.int64), np.arange(cols, dtype=np.int64),
                         indexing="ij")
    vid = (ii * cols + jj).ravel()
    right = (ii * cols + (jj + 1) % cols).ravel()
    down = (((ii + 1) % rows) * cols + jj).ravel()
    return csr_from_edges(rows * cols, np.concatenate([vid, vid]),
                          np.concatenate([right, down]), f"torus{rows}x{cols}")


def random_graph(n: int, m: int, seed: int) -> CSRGraph:
    """m uniform random vertex pairs (self-loops and repeats dropped)."""
    rng = np.random.default_rng(seed)
    return csr_from_edges(n, rng.integers(0, n, m), rng.integers(0, n, m), f"rand{n}_{m}_s{seed}")


# ---------------------------------------------------------------- sources
def max_degree_vertex(g: CSRGraph) -> int:
    """Highest-degree vertex, ties to the lowest ID."""
    return int(np.argmax(g.degrees)) if g.n else 0


def random_source(g: CSRGraph, seed: int) -> int:
    return int(np.random.default_rng(seed).integers(0, g.n))


def random_nonisolated_sources(g: CSRGraph, count: int, seed: int) -> np.ndarray:
    cand = np.flatnonzero(g.degrees > 0)
    if cand.size == 0:
        cand = np.arange(g.n)
    return np.random.default_rng(seed).choice(cand, size=count).astype(np.int64)


def describe(g: CSRGraph) -> dict:
    deg = g.degrees
    return {"name": g.name, "n": g.n, "m": g.m,
            "max_degree": int(deg.max()) if g.n else 0,
            "isolated": int((deg == 0).sum()),
            "avg_degree": float(g.m / g.n) if g.n else 0.0}


if __name__ == "__main__":  # pragma: no cover - manual inspection
    import sys
    import time
    t = time.time()
    which = sys.argv[1] if len(sys.argv) > 1 else "rmat16"
    if which.startswith("rmat"):
        s = int(which[4:])
        g = rmat_graph(s, 8 if s == 16 else 16, seed=1, permute_seed=None if s == 16 else 2)
    else:
        g = grid_graph(int(which[4:]))
    print(describe(g), f"{time.time() - t:.1f}s")


# ---------------------------------------------------------------- batches (device-side generation)
# The batched workload has hundreds of graphs and ~10^9 edges; these helpers
# draw them with torch on a given device (a seeded torch.Generator), so the
# same code serves small CPU-side test batches and the full GPU-side one.
def _torch_csr(n, src, dst):
    import torch
    keep = src != dst
    src, dst = src[keep], dst[keep]
    key = torch.unique(torch.cat([src * n + dst, dst * n + src]))
    s = torch.div(key, n, rounding_mode="floor")
    cols = (key - s * n).to(torch.int32)
    offsets = torch.zeros(n + 1, dtype=torch.int64, device=key.device)
    offsets[1:] = torch.cumsum(torch.bincount(s, minlength=n), 0)
    return offsets, cols


def rmat_csr_torch(scale, edge_factor, seed, device="cpu", a=0.57, b=0.19, c=0.19):
    """R-MAT graph (same quadrant rule as rmat_graph) drawn with torch; returns
    (offsets int64, cols int32) tensors on `device`."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    n = 1 << scale
    m = int(edge_factor) << int(scale)
    src = torch.zeros(m, dtype=torch.int64, device=device)
    dst = torch.zeros(m, dtype=torch.int64, device=device)
    ab, abc = a + b, a + b + c
    for level in range(scale):
        u = torch.rand(m, generator=gen, device=device)
        src |= (u >= ab).long() << level
        dst |= (((u >= a) & (u < ab)) | (u >= abc)).long() << level
    return _torch_csr(n, src, dst)


def _largest_component_csr(offsets, cols):
    """Largest connected component of a symmetric CSR (torch tensors), vertex
    ids relabelled in increasing order; computed on the host with scipy."""
    import torch
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    dev = offsets.device
    o = offsets.cpu().numpy()
    c = cols.cpu().numpy()
    n = o.size - 1
    mat = sp.csr_matrix((np.ones(c.size, dtype=np.int8), c, o), shape=(n, n))
    _, labels = connected_components(mat, directed=False)
    keep = labels == np.argmax(np.bincount(labels))
    new_id = np.cumsum(keep) - 1
    deg = np.diff(o)
    c_keep = new_id[c[np.repeat(keep, deg)]].astype(np.int32)
    o_keep = np.zeros(int(keep.sum()) + 1, dtype=np.int64)
    o_keep[1:] = np.cumsum(deg[keep])
    return torch.from_numpy(o_keep).to(dev), torch.from_numpy(c_keep).to(dev)


def grid_csr_torch(side, seed, device="cpu", delete_frac=0.2, diag_frac=0.01, lcc=False):
    """Perturbed grid (same recipe as grid_graph; the largest-component step
    only with `lcc`) drawn with torch; returns (offsets int64, cols int32)."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    n = side * side
    idx = torch.arange(n, dtype=torch.int64, device=device)
    i, j = idx // side, idx % side
    hu = idx[j < side - 1]
    vu = idx[i < side - 1]
    src = torch.cat([hu, vu])
    dst = torch.cat([hu + 1, vu + side])
    m = src.numel()
    ndel = int(round(delete_frac * m))
    if ndel:
        keep = torch.randperm(m, generator=gen, device=device)[ndel:]
        src, dst = src[keep], dst[keep]
    ndiag = int(round(diag_frac * n))
    if ndiag:
        start = torch.randint(0, n, (ndiag,), generator=gen, device=device)
        direction = torch.randint(0, 4, (ndiag,), generator=gen, device=device)
        di = torch.where(direction < 2, -1, 1)
        dj = torch.where(direction % 2 == 0, -1, 1)
        ti, tj = start // side + di, start % side + dj
        ok = (ti >= 0) & (ti < side) & (tj >= 0) & (tj < side)
        src = torch.cat([src, start[ok]])
        dst = torch.cat([dst, (ti * side + tj)[ok]])
    offsets, cols = _torch_csr(n, src, dst)
    return _largest_component_csr(offsets, cols) if lcc else (offsets, cols)


def nonisolated_sources_torch(offsets, count, seed):
    """`count` sources drawn uniformly (with replacement) over the vertices of
    degree > 0 of a CSR given as torch offsets; numpy int64 array."""
    deg = (offsets[1:] - offsets[:-1]).cpu().numpy()
    cand = np.flatnonzero(deg > 0)
    if cand.size == 0:
        cand = np.arange(deg.size)
    return np.random.default_rng(seed).choice(cand, size=count).astype(np.int64)


@dataclasses.dataclass
class BatchWorkload:
    """Union graph of many instances plus each instance's own CSR.

    instances: list of (app, vertex_begin, vertex_end, global_source);
    local: list of (offsets, cols, local_source) per instance (torch tensors)."""
    n: int
    offsets: object
    cols: object
    instances: list
    local: list
    kinds: list


def batch_workload(n_graphs=640, n_pagerank=128, scales=(10, 18), edge_factors=(4, 32),
                   grid_sides=(32, 1024), seed=4, device="cpu") -> BatchWorkload:
    """Half R-MAT graphs (integer scale uniform in `scales`, edge factor
    uniform in `edge_factors`), half perturbed grids (side log-uniform in
    `grid_sides`), interleaved; `n_pagerank` instances chosen uniformly are
    PageRank, the rest BFS from a uniform non-isolated vertex."""
    import torch
    rng = np.random.default_rng(seed)
    apps = np.full(n_graphs, 1, dtype=np.int64)  # 1 = BFS, 2 = PageRank
    apps[rng.choice(n_graphs, size=n_pagerank, replace=False)] = 2
    offs_parts, cols_parts, instances, local, kinds = [], [], [], [], []
    vbase = ebase = 0
    for k in range(n_graphs):
        gseed = int(rng.integers(0, 2 ** 31 - 1))
        if k % 2 == 0:
            scale = int(rng.integers(scales[0], scales[1] + 1))
            ef = int(rng.integers(edge_factors[0], edge_factors[1] + 1))
            o, c = rmat_csr_torch(scale, ef, gseed, device=device)
            kinds.append(f"rmat{scale}_ef{ef}")
        else:
            side = int(round(np.exp(rng.uniform(np.log(grid_sides[0]), np.log(grid_sides[1])))))
            o, c = grid_csr_torch(side, gseed, device=device)
            kinds.append(f"grid{side}")
        n = o.numel() - 1
        deg = o[1:] - o[:-1]
        cand = torch.nonzero(deg > 0).flatten()
        pick = int(rng.integers(0, max(int(cand.numel()), 1)))
        src = int(cand[pick].item()) if cand.numel() else 0
        local.append((o, c, src))
        offs_parts.append(o[:-1] + ebase)
        cols_parts.append(c + vbase)
        instances.append((int(apps[k]), vbase, vbase + n, vbase + src))
        vbase += n
        ebase += int(c.numel())
    offs_parts.append(torch.tensor([ebase], dtype=torch.int64, device=device))
    return BatchWorkload(vbase, torch.cat(offs_parts), torch.cat(cols_parts).to(torch.int32),
                         instances, local, kinds)
