"""Seeded synthetic inputs for the independent-set tensor-network workloads.

This module only draws graphs and vertex weights.  It contains none of the
contraction arithmetic, so both the CPU oracle (``oracle/``) and the GPU path
use it without sharing any of the method's code.

Graph classes follow the ones the paper evaluates (Sec. 2, the graph zoo; Sec. 6):

* ``petersen()``            -- the Petersen graph in its textbook labelling
* ``square_lattice(L)``     -- the full L x L 4-neighbour grid
* ``kings_subgraph(L, p)``  -- L x L sites, each kept with probability p, edges
                               between kept sites at Chebyshev distance 1
* ``random_regular(n, d)``  -- uniform simple d-regular graph (pairing model
                               with rejection)
* plus small closed-form families (path, cycle, complete, complete bipartite,
  empty, G(n, p)) used to pin the oracle.

The random stream is SplitMix64 (Steele, Lea, Flood 2014), written out here so
every instance is reproducible byte for byte on any host.  The paper's own
instances came from Julia's RNG and cannot be reproduced; they are not needed.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np

_MASK64 = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 generator: state += golden gamma, then a 3-step mixer."""

    def __init__(self, seed: int):
        self.state = seed & _MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
        return z ^ (z >> 31)

    def uniform(self) -> float:
        """Double in [0, 1) with 53 random bits."""
        return (self.next_u64() >> 11) * (1.0 / (1 << 53))

    def below(self, n: int) -> int:
        """Unbiased integer in [0, n) by rejection."""
        if n <= 0:
            raise ValueError("below(n) needs n > 0")
        limit = (1 << 64) - ((1 << 64) % n)
        while True:
            x = self.next_u64()
            if x < limit:
                return x % n

    def shuffle(self, xs: list) -> None:
        for i in range(len(xs) - 1, 0, -1):
            j = self.below(i + 1)
            xs[i], xs[j] = xs[j], xs[i]


def _stream(seed: int, salt: int) -> SplitMix64:
    # decorrelate the streams used for graph structure and for weights
    r = SplitMix64(seed ^ (salt * 0xD1B54A32D192ED03 & _MASK64))
    r.next_u64()
    return r


@dataclasses.dataclass
class Graph:
    """Undirected simple graph with 0-based vertices and optional weights."""

    nv: int
    edges: np.ndarray  # int32 [m, 2], u < v, sorted, no duplicates
    weights: Optional[np.ndarray] = None  # float32 [nv] or None (unit weights)
    name: str = ""

    @property
    def ne(self) -> int:
        return int(self.edges.shape[0])

    def with_weights(self, w: Optional[np.ndarray]) -> "Graph":
        if w is not None:
            w = np.ascontiguousarray(w, dtype=np.float32)
            if w.shape != (self.nv,):
                raise ValueError("weights must have one entry per vertex")
        return Graph(self.nv, self.edges, w, self.name)

    def adjacency(self) -> List[List[int]]:
        adj: List[List[int]] = [[] for _ in range(self.nv)]
        for u, v in self.edges.tolist():
            adj[u].append(v)
            adj[v].append(u)
        return adj


def _make(nv: int, pairs: Sequence[Tuple[int, int]], name: str) -> Graph:
    es = sorted({(min(u, v), max(u, v)) for u, v in pairs if u != v})
    arr = np.array(es, dtype=np.int32).reshape(-1, 2)
    return Graph(nv, arr, None, name)


def petersen() -> Graph:
    """Outer cycle 0-1-2-3-4-0, spokes i-(i+5), inner pentagram 5-7-9-6-8-5.

    With vertex k printed as character k, this is the labelling under which the
    paper's five maximum independent sets (Sec. 5, ConfigsMax example) are the
    maximum independent sets.
    """
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5, 7), (7, 9), (9, 6), (6, 8), (8, 5)]
    return _make(10, outer + spokes + inner, "petersen")


def path(n: int) -> Graph:
    return _make(n, [(i, i + 1) for i in range(n - 1)], f"path{n}")


def cycle(n: int) -> Graph:
    if n < 3:
        raise ValueError("cycle needs n >= 3")
    return _make(n, [(i, (i + 1) % n) for i in range(n)], f"cycle{n}")


def complete(n: int) -> Graph:
    return _make(n, [(i, j) for i in range(n) for j in range(i + 1, n)], f"K{n}")


def complete_bipartite(a: int, b: int) -> Graph:
    return _make(a + b, [(i, a + j) for i in range(a) for j in range(b)], f"K{a},{b}")


def empty(n: int) -> Graph:
    return _make(n, [], f"empty{n}")


def star(n_leaves: int) -> Graph:
    return _make(n_leaves + 1, [(0, i + 1) for i in range(n_leaves)], f"star{n_leaves}")


def disjoint_union(g: Graph, h: Graph) -> Graph:
    off = g.nv
    pairs = [tuple(e) for e in g.edges.tolist()] + [(u + off, v + off) for u, v in h.edges.tolist()]
    out = _make(g.nv + h.nv, pairs, f"{g.name}+{h.name}")
    if g.weights is not None or h.weights is not None:
        gw = g.weights if g.weights is not None else np.ones(g.nv, np.float32)
        hw = h.weights if h.weights is not None else np.ones(h.nv, np.float32)
        out = out.with_weights(np.concatenate([gw, hw]))
    return out


def induced(g: Graph, keep: Sequence[int]) -> Graph:
    """The subgraph induced by the vertices in keep, relabelled 0.. in keep's
    order (weights follow their vertices)."""
    pos = {int(v): k for k, v in enumerate(keep)}
    pairs = [(pos[u], pos[v]) for u, v in g.edges.tolist() if u in pos and v in pos]
    out = _make(len(pos), pairs, f"{g.name}[{len(pos)}]")
    if g.weights is not None:
        out = out.with_weights(np.asarray([g.weights[int(v)] for v in keep], np.float32))
    return out


def square_lattice(L: int) -> Graph:
    """Full L x L grid, vertex (r, c) -> r*L + c, 4-neighbour edges."""
    pairs = []
    for r in range(L):
        for c in range(L):
            v = r * L + c
            if c + 1 < L:
                pairs.append((v, v + 1))
            if r + 1 < L:
                pairs.append((v, v + L))
    return _make(L * L, pairs, f"square{L}")


def grid(rows: int, cols: int) -> Graph:
    """Full rows x cols grid, vertex (r, c) -> r*cols + c, 4-neighbour edges."""
    pairs = []
    for r in range(rows):
        for c in range(cols):
            v = r * cols + c
            if c + 1 < cols:
                pairs.append((v, v + 1))
            if r + 1 < rows:
                pairs.append((v, v + cols))
    return _make(rows * cols, pairs, f"grid{rows}x{cols}")


def fullerene() -> Graph:
    """The C60 buckyball of the Sec. 6.4 example: the 60 vertices of a truncated
    icosahedron (all cyclic coordinate rotations and sign changes of
    (0, 1, 3phi), (1, 2 + phi, 2 phi), (phi, 2, 2 phi + 1), phi the golden
    ratio), joined when at most sqrt(5) apart (its 90 edges, all of length 2)."""
    import math

    phi = (1.0 + math.sqrt(5.0)) / 2.0
    pts = []
    for base in ((0.0, 1.0, 3 * phi), (1.0, 2 + phi, 2 * phi), (phi, 2.0, 2 * phi + 1)):
        for r in range(3):
            a, b, c = base[r % 3], base[(r + 1) % 3], base[(r + 2) % 3]
            for sa in (1, -1):
                for sb in (1, -1):
                    for sc in (1, -1):
                        q = (sa * a, sb * b, sc * c)
                        if not any(max(abs(x - y) for x, y in zip(q, o)) < 1e-9 for o in pts):
                            pts.append(q)
    edges = [(i, j) for i in range(len(pts)) for j in range(i + 1, len(pts))
             if math.dist(pts[i], pts[j]) <= math.sqrt(5.0) + 1e-9]
    return _make(len(pts), edges, "fullerene")


def kings_subgraph(L: int, p: float, seed: int) -> Graph:
    """King's subgraph: keep each site of an L x L grid with probability p.

    Kept sites are numbered in row-major order; two kept sites are adjacent
    when their Chebyshev distance is 1 (horizontal, vertical, diagonal).
    """
    rng = _stream(seed, 1)
    keep = np.zeros((L, L), dtype=bool)
    for r in range(L):
        for c in range(L):
            keep[r, c] = rng.uniform() < p
    ids = -np.ones((L, L), dtype=np.int64)
    nv = 0
    for r in range(L):
        for c in range(L):
            if keep[r, c]:
                ids[r, c] = nv
                nv += 1
    pairs = []
    for r in range(L):
        for c in range(L):
            if not keep[r, c]:
                continue
            for dr, dc in ((0, 1), (1, -1), (1, 0), (1, 1)):
                rr, cc = r + dr, c + dc
                if 0 <= rr < L and 0 <= cc < L and keep[rr, cc]:
                    pairs.append((int(ids[r, c]), int(ids[rr, cc])))
    return _make(nv, pairs, f"ksg{L}@{p}s{seed}")


def random_regular(n: int, d: int, seed: int, max_tries: int = 100000) -> Graph:
    """Uniform simple d-regular graph via the pairing (configuration) model.

    Points are paired by a seeded shuffle; a pairing with a loop or a repeated
    edge is rejected and redrawn, which makes the accepted graph uniform.
    """
    if (n * d) % 2 != 0 or d >= n:
        raise ValueError("need n*d even and d < n")
    rng = _stream(seed, 2)
    for _ in range(max_tries):
        pts = [v for v in range(n) for _ in range(d)]
        rng.shuffle(pts)
        seen = set()
        ok = True
        for a in range(0, len(pts), 2):
            u, v = pts[a], pts[a + 1]
            if u == v:
                ok = False
                break
            e = (min(u, v), max(u, v))
            if e in seen:
                ok = False
                break
            seen.add(e)
        if ok:
            return _make(n, list(seen), f"reg{d}n{n}s{seed}")
    raise RuntimeError("pairing model did not produce a simple graph")


def gnp(n: int, p: float, seed: int) -> Graph:
    rng = _stream(seed, 3)
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.uniform() < p]
    return _make(n, pairs, f"gnp{n}p{p}s{seed}")


def dyadic_weights(n: int, seed: int, bits: int = 14) -> np.ndarray:
    """Weights k / 2^bits with k uniform in [0, 2^bits), as float32.

    Every partial sum of up to a few thousand such weights is exact in FP32,
    so tropical results do not depend on the order of additions.
    """
    rng = _stream(seed, 4)
    return np.array([rng.below(1 << bits) / float(1 << bits) for _ in range(n)], dtype=np.float32)


def uniform_weights(n: int, seed: int) -> np.ndarray:
    """Generic FP32 weights uniform in [0, 1) (24 random mantissa bits)."""
    rng = _stream(seed, 5)
    return np.array([(rng.next_u64() >> 40) * (1.0 / (1 << 24)) for _ in range(n)], dtype=np.float32)


def integer_weights(n: int, seed: int, lo: int = 1, hi: int = 4) -> np.ndarray:
    """Small integer weights in [lo, hi], as float32 (exact)."""
    rng = _stream(seed, 6)
    return np.array([lo + rng.below(hi - lo + 1) for _ in range(n)], dtype=np.float32)


def poisson_arrivals(n_jobs: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process with the given rate."""
    rng = _stream(seed, 7)
    t = 0.0
    out = np.empty(n_jobs, dtype=np.float64)
    for i in range(n_jobs):
        u = rng.uniform()
        t += -np.log1p(-u) / rate
        out[i] = t
    return out


def job_mix(n_jobs: int, seed: int, n_lo: int = 40, n_hi: int = 200,
            semirings: Sequence[str] = ("tropical_i32", "counting_tropical", "partition_f32")):
    """Served-stream job list: (n, graph seed, semiring) per job.

    n is uniform over the even integers in [n_lo, n_hi] (a 3-regular graph
    needs an even vertex count); the semiring is uniform over ``semirings``.
    """
    rng = _stream(seed, 8)
    evens = list(range(n_lo + (n_lo & 1), n_hi + 1, 2))
    jobs = []
    for j in range(n_jobs):
        n = evens[rng.below(len(evens))]
        sr = semirings[rng.below(len(semirings))]
        jobs.append((n, int(rng.next_u64() & 0x7FFFFFFF), sr))
    return jobs
