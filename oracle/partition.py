"""Reference graph partitioner -- TEST INFRASTRUCTURE ONLY.

A plain Python statement of the recursive bisection the library offers for
matrices without a geometric split (the method takes the partition as an input
from a graph partitioner, Sec. 2.1).  Shares no code with the library.

Definition:
  * a vertex set with q parts to form is cut after the first
    round(|set| * floor(q/2) / q) vertices (halves rounded up) of a
    breadth-first order of its induced subgraph; the first piece gets
    floor(q/2) parts and the lower ids, the second q - floor(q/2);
  * the breadth-first order starts at a pseudo-peripheral vertex: begin at the
    lowest-numbered vertex of the set; while a BFS from the lowest-numbered
    vertex of the deepest level has more levels, move there (at most 8 moves);
  * neighbours are visited in ascending order, the diagonal is ignored, and
    vertices not reached are appended by BFS from the lowest unreached vertex.
"""
from __future__ import annotations

from collections import deque

import numpy as np


def _bfs(adj, inset, root, seen, order):
    """BFS from root inside the set; appends to order, returns {vertex: level} of this search."""
    lev = {root: 0}
    seen.add(root)
    order.append(root)
    q = deque([root])
    while q:
        u = q.popleft()
        for v in adj[u]:
            if v != u and v in inset and v not in seen:
                seen.add(v)
                lev[v] = lev[u] + 1
                order.append(v)
                q.append(v)
    return lev


def _order(adj, vs):
    inset = set(vs)
    root = min(vs)
    lev = _bfs(adj, inset, root, set(), [])
    depth = max(lev.values())
    for _ in range(8):
        far = min(v for v, l in lev.items() if l == depth)
        lev2 = _bfs(adj, inset, far, set(), [])
        d2 = max(lev2.values())
        if d2 <= depth:
            break
        root, lev, depth = far, lev2, d2
    seen, order = set(), []
    _bfs(adj, inset, root, seen, order)
    for v in sorted(vs):
        if v not in seen:
            _bfs(adj, inset, v, seen, order)
    return order


def partition_graph(A, p: int) -> np.ndarray:
    n = A.n
    rp, ci = np.asarray(A.rowptr), np.asarray(A.col)
    adj = [ci[rp[i]:rp[i + 1]].tolist() for i in range(n)]
    part = np.full(n, -1, np.int32)

    def split(vs, q, base):
        if q == 1 or len(vs) <= 1:
            part[vs] = base
            return
        order = _order(adj, vs)
        q1 = q // 2
        t = (len(vs) * q1 * 2 + q) // (2 * q)
        split(sorted(order[:t]), q1, base)
        split(sorted(order[t:]), q - q1, base + q1)

    split(list(range(n)), p, 0)
    return part
