"""Cluster tree for HSS compression (oracle).

Follows Sec. 2.1 (HSS representation): a binary tree numbered level by
level, top-down, from 0 at the root; every node owns a contiguous index
range I_tau of the permuted index set, the two children partition it, and
the same tree serves rows and columns.  The paper leaves the splitting
rule to the user; the reading used here:

* a node with m > leaf_size indices splits into floor(m/2) (left) and the
  rest (right);
* 'bisect': plain index bisection, permutation = identity;
* 'rcb': recursive coordinate bisection, split axis = the axis of largest
  extent of the node's points (ties -> lowest axis);
* 'kd': split axis = depth mod 3;
* points are ordered by (coordinate, original index); inside a leaf by
  original index;
* BFS numbering, left child before right child.

Plain Python loops; meant for reference and tests.
"""
from __future__ import annotations

from collections import deque
from dataclasses import dataclass

import numpy as np


@dataclass
class Tree:
    n: int
    lo: np.ndarray      # int64[num_nodes]
    hi: np.ndarray      # int64[num_nodes]
    left: np.ndarray    # int64[num_nodes], -1 for leaves
    right: np.ndarray   # int64[num_nodes], -1 for leaves
    parent: np.ndarray  # int64[num_nodes], -1 for the root
    level: np.ndarray   # int64[num_nodes], 0 at the root
    perm: np.ndarray    # int64[n]: permuted position i holds original index perm[i]

    @property
    def num_nodes(self) -> int:
        return len(self.lo)

    def is_leaf(self, t: int) -> bool:
        return self.left[t] < 0

    def size(self, t: int) -> int:
        return int(self.hi[t] - self.lo[t])

    def levels(self) -> int:
        return int(self.level.max()) + 1


def build_tree(n: int, leaf_size: int, points: np.ndarray | None = None,
               method: str = "bisect") -> Tree:
    if n < 1 or leaf_size < 1:
        raise ValueError("n and leaf_size must be positive")
    if method != "bisect":
        if points is None or points.shape != (n, 3):
            raise ValueError("rcb/kd need an (n,3) point array")
        if not np.all(np.isfinite(points)):
            raise ValueError("non-finite point coordinates")
    lo, hi, left, right, parent, level = [], [], [], [], [], []
    members = []   # original indices owned by each node, in order
    queue = deque()
    lo.append(0); hi.append(n); left.append(-1); right.append(-1)
    parent.append(-1); level.append(0)
    members.append(list(range(n)))
    queue.append(0)
    while queue:
        t = queue.popleft()
        idx = members[t]
        m = len(idx)
        if m <= leaf_size:
            members[t] = sorted(idx)
            continue
        if method == "bisect":
            ordered = idx
        else:
            if method == "rcb":
                best_axis, best_ext = 0, None
                for a in range(3):
                    vals = [points[i, a] for i in idx]
                    ext = max(vals) - min(vals)
                    if best_ext is None or ext > best_ext:
                        best_axis, best_ext = a, ext
                axis = best_axis
            elif method == "kd":
                axis = level[t] % 3
            else:
                raise ValueError("unknown tree method " + method)
            ordered = sorted(idx, key=lambda i: (points[i, axis], i))
        half = m // 2
        for part, (a, b) in ((0, (0, half)), (1, (half, m))):
            c = len(lo)
            lo.append(lo[t] + a); hi.append(lo[t] + b)
            left.append(-1); right.append(-1)
            parent.append(t); level.append(level[t] + 1)
            members.append(list(ordered[a:b]))
            if part == 0:
                left[t] = c
            else:
                right[t] = c
            queue.append(c)
    perm = np.empty(n, dtype=np.int64)
    for t in range(len(lo)):
        if left[t] < 0:
            perm[lo[t]:hi[t]] = members[t]
    arr = lambda v: np.asarray(v, dtype=np.int64)
    return Tree(n, arr(lo), arr(hi), arr(left), arr(right), arr(parent), arr(level), perm)
