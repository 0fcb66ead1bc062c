"""Explicit contraction trees whose intermediates reach 2^30 entries on
graphs of small treewidth (test inputs, not part of the library).

A tree is given in the format of ``tn_plan_from_tree``: leaves are lists of
factor codes (edge id >= 0, vertex tensor of v as -v-1), inner node t has id
nleaf + t and children with smaller ids, the last node is the root.  The
intermediates follow the einsum rule of the paper's Sec. 4.1 (an index stays
while it occurs outside the subtree), so the rank of a subtree is the number
of its vertices that also occur in tensors outside it.

``three_row_gemm_tree(W, m)`` works on the 3 x W grid (rows r = 0, 1, 2,
vertex (r, c) = r*W + c):

* X: the row-0 chain, then the vertical edges (0,c)-(1,c) for c < m, one at a
  time; X holds row 0 from column m on and row 1 below column m (W indices).
* Y: the row-1 edges left of column m and the vertical edges (1,c)-(2,c) for
  c < m (2m + 1 indices).
* C = X (x) Y sums the m vertices (1, c < m): i = row 0 from column m on,
  j = (1, m) and (2, c < m), k = m, so |C| = 2^(W+1) entries after a
  contraction of 2^(W+1+m) semiring operations.
* The rest of the grid is then absorbed one edge at a time, column by
  column, so every later intermediate has at most W + 1 indices.

The graph's treewidth is 3, so the oracle's variable elimination solves it
exactly in every algebra: an independent check of a contraction whose
largest tensors are 2^(W+1) entries.
"""
from __future__ import annotations

from typing import Dict, List, Tuple


class TreeBuilder:
    def __init__(self, edges):
        self.eid: Dict[Tuple[int, int], int] = {(int(u), int(v)): k for k, (u, v) in enumerate(edges.tolist())}
        self.leaves: List[List[int]] = []
        self.nodes: List[Tuple[tuple, tuple]] = []
        self.vertex_done = set()

    def edge(self, u: int, v: int) -> tuple:
        a, b = min(u, v), max(u, v)
        fac = [self.eid[(a, b)]]
        for x in (a, b):  # each vertex tensor rides with the first edge that holds it
            if x not in self.vertex_done:
                self.vertex_done.add(x)
                fac.append(-x - 1)
        self.leaves.append(fac)
        return ("L", len(self.leaves) - 1)

    def join(self, a: tuple, b: tuple) -> tuple:
        self.nodes.append((a, b))
        return ("N", len(self.nodes) - 1)

    def chain(self, items) -> tuple:
        items = list(items)
        acc = items[0]
        for x in items[1:]:
            acc = self.join(acc, x)
        return acc

    def export(self):
        nl = len(self.leaves)

        def ident(x):
            return x[1] if x[0] == "L" else nl + x[1]

        left = [ident(a) for a, _ in self.nodes]
        right = [ident(b) for _, b in self.nodes]
        return self.leaves, left, right


def three_row_gemm_tree(W: int, m: int, edges):
    """Leaves, left, right of the tree described in the module docstring."""
    def vid(r, c):
        return r * W + c

    t = TreeBuilder(edges)
    # X: row-0 chain, then the verticals (0,c)-(1,c) for c < m
    x = t.chain([t.edge(vid(0, c), vid(0, c + 1)) for c in range(W - 1)])
    for c in range(m):
        x = t.join(x, t.edge(vid(0, c), vid(1, c)))
    # Y: row-1 edges left of column m and verticals (1,c)-(2,c), c < m
    ys = []
    for c in range(m):
        ys.append(t.edge(vid(1, c), vid(2, c)))
        ys.append(t.edge(vid(1, c), vid(1, c + 1)))
    y = t.chain(ys)
    acc = t.join(x, y)  # the 2^(W+1)-entry contraction
    # row 2 left of column m
    for c in range(m):
        acc = t.join(acc, t.edge(vid(2, c), vid(2, c + 1)))
    # the remaining columns, left to right
    for c in range(m, W):
        acc = t.join(acc, t.edge(vid(0, c), vid(1, c)))
        acc = t.join(acc, t.edge(vid(1, c), vid(2, c)))
        if c + 1 < W:
            acc = t.join(acc, t.edge(vid(1, c), vid(1, c + 1)))
            acc = t.join(acc, t.edge(vid(2, c), vid(2, c + 1)))
    assert len(t.vertex_done) == 3 * W and sum(len(l) for l in t.leaves) == len(edges) + 3 * W
    return t.export()
