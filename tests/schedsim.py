"""Test-only schedule simulator (CPU): the asynchronous task semantics of the
worker kernel, run with every task advanced one neighbour at a time in a
random interleaving with every other task in flight, and tasks started in a
random order rather than FIFO.

It is neither the oracle (which fixes what the results are) nor GPU code: it
shows that the update rules give order-independent results (BFS depths
exact, PageRank within its bound, colourings valid) under schedules far more
scrambled than a GPU's, which the tests check against the oracle.

Rules simulated (paper section 5):
- BFS (Algorithm 2): a task carries the depth its pusher set (low 16 bits); a
  stale duplicate is dropped at start; each neighbour is relaxed with an
  atomic minimum and pushed when it improved.
- PageRank (Algorithm 4, threshold-crossing enqueue): a task takes its vertex's
  whole residue, adds it to the rank and pushes damping*residue/degree to each
  neighbour, enqueueing a neighbour exactly when its residue crosses epsilon.
- Colouring (Algorithm 6 with the rank rule and the ordered class): an
  assignment takes the first colour no outranking neighbour holds (class
  vertices wait until every outranking neighbour is coloured); a check makes
  the lower-ranked endpoint of a conflict recolour and counts a class vertex
  off its lower-ranked class neighbours' waits.
"""
from __future__ import annotations

import numpy as np


def _adj(g):
    off = np.asarray(g.offsets, dtype=np.int64)
    cols = np.asarray(g.cols, dtype=np.int64)
    return [cols[off[v]:off[v + 1]].tolist() for v in range(g.n)]


class _Sched:
    """Tasks in flight are generators; a step advances one of them (chosen at
    random) by one neighbour, or starts a random queued task."""

    def __init__(self, rng, max_inflight: int):
        self.rng = rng
        self.queue: list = []
        self.running: list = []
        self.max_inflight = max_inflight
        self.started = 0

    def push(self, task):
        self.queue.append(task)

    def run(self, start):
        while self.queue or self.running:
            if self.queue and (not self.running or len(self.running) < self.max_inflight
                               and self.rng.random() < 0.5):
                i = int(self.rng.integers(len(self.queue)))
                self.queue[i], self.queue[-1] = self.queue[-1], self.queue[i]
                gen = start(self.queue.pop())
                self.started += 1
                if gen is not None:
                    self.running.append(gen)
                continue
            i = int(self.rng.integers(len(self.running)))
            try:
                next(self.running[i])
            except StopIteration:
                self.running[i] = self.running[-1]
                self.running.pop()


def bfs(g, source: int, seed: int, max_inflight: int = 16) -> np.ndarray:
    adj = _adj(g)
    unreached = 0xFFFFFFFF
    depth = [unreached] * g.n
    depth[source] = 0
    s = _Sched(np.random.default_rng(seed), max_inflight)

    def start(task):
        v, tag = task
        d = depth[v]
        if (d & 0xFFFF) != tag:
            return None  # a newer push expands v

        def body():
            nd = d + 1
            for w in adj[v]:
                yield
                if nd < depth[w]:  # atomic minimum, pushed when it lowered the depth
                    old = depth[w]
                    depth[w] = min(old, nd)
                    if nd < old:
                        s.push((w, nd & 0xFFFF))
        return body()

    s.push((source, 0))
    s.run(start)
    return np.array([-1 if d == unreached else d for d in depth], dtype=np.int64)


def pagerank(g, damping: float, eps: float, seed: int, max_inflight: int = 16):
    adj = _adj(g)
    deg = [len(a) for a in adj]
    rank = [1.0 - damping] * g.n
    residue = [(1.0 - damping) * damping * sum(1.0 / deg[u] for u in adj[v]) for v in range(g.n)]
    s = _Sched(np.random.default_rng(seed), max_inflight)

    def start(v):
        r = residue[v]  # atomic exchange with zero
        residue[v] = 0.0
        if not r > 0.0:
            return None
        rank[v] += r
        if deg[v] == 0:
            return None

        def body():
            delta = damping * r / deg[v]
            for w in adj[v]:
                yield
                old = residue[w]
                residue[w] = old + delta
                if old <= eps < old + delta:
                    s.push(w)
        return body()

    for v in range(g.n):
        s.push(v)
    s.run(start)
    return np.array(rank), np.array(residue), s.started


def color(g, key: np.ndarray, order: int, seed: int, max_inflight: int = 16) -> np.ndarray:
    """`key`: the rank keys (degree high, priority low); `order` > 0: degree of
    the ordered class."""
    adj = _adj(g)
    deg = [len(a) for a in adj]
    k = [int(x) for x in key]
    colour = [-1] * g.n
    queued = [1] * g.n

    def up(w, v):  # w outranks v
        return k[w] > k[v] if k[w] != k[v] else w > v

    def ordered(v):
        return order > 0 and (k[v] >> 16) >= order

    wait = [sum(1 for w in adj[v] if w != v and up(w, v)) if ordered(v) else 0 for v in range(g.n)]
    s = _Sched(np.random.default_rng(seed), max_inflight)

    def start(task):
        v, kind = task
        if kind == 0:  # assign
            if ordered(v) and (wait[v] != 0 or colour[v] >= 0):
                return None
            queued[v] = 0

            def assign():
                seen = set()
                for w in adj[v]:
                    yield
                    if w != v and up(w, v) and colour[w] >= 0:
                        seen.add(colour[w])
                c = 0
                while c in seen:
                    c += 1
                if ordered(v):
                    if colour[v] >= 0:
                        return
                    colour[v] = c
                    yield from check(v)
                else:
                    colour[v] = c
                    s.push((v, 1))
            return assign()
        return check(v)

    def check(v):
        c = colour[v]
        again = False
        for w in adj[v]:
            yield
            if w == v:
                continue
            if colour[w] == c:
                if up(w, v):
                    again = True
                elif queued[w] == 0:
                    queued[w] = 1
                    s.push((w, 0))
            elif not up(w, v) and ordered(v) and ordered(w):
                wait[w] -= 1
                if wait[w] == 0:
                    s.push((w, 0))
        if again and queued[v] == 0:
            queued[v] = 1
            s.push((v, 0))

    for v in range(g.n):
        s.push((v, 0))
    s.run(start)
    return np.array(colour, dtype=np.int64)
