"""Brute-force UniFrac for tiny trees (test oracle only).

Independent of the postorder pass in ``oracle.unifrac``: for every non-root
node v, the set of tips under v is found by walking parent pointers up from
each tip and recording every node passed.  The distances are then the plain
sums of the definitions (paper section II names the unweighted and the
weighted-normalized variants), using Python floats and loops.
Cost O(M * tips * depth + N^2 * M); meant for trees of a few dozen nodes.
"""
from __future__ import annotations

from typing import Dict, List, Set


def _tips_under(parent: List[int]) -> Dict[int, Set[int]]:
    m = len(parent)
    has_child = [False] * m
    for v in range(m):
        if parent[v] >= 0:
            has_child[parent[v]] = True
    under: Dict[int, Set[int]] = {v: set() for v in range(m)}
    for t in range(m):
        if has_child[t]:
            continue
        v = t
        steps = 0
        while v >= 0:
            under[v].add(t)
            v = parent[v]
            steps += 1
            if steps > m:
                raise ValueError("cycle")
    return under


def dm(parent, length, rows, variant: str) -> List[float]:
    """Condensed distances for samples given as dicts {tip node id: count}."""
    parent = [int(p) for p in parent]
    length = [float(x) for x in length]
    under = _tips_under(parent)
    branches = [v for v in range(len(parent)) if parent[v] >= 0]
    emb = []
    for row in rows:
        total = sum(row.values())
        c = {v: sum(row.get(t, 0) for t in under[v]) for v in branches}
        emb.append(({v: c[v] / total for v in branches},
                    {v: 1.0 if c[v] > 0 else 0.0 for v in branches}))
    out = []
    n = len(rows)
    for i in range(n):
        for j in range(i + 1, n):
            num = 0.0
            den = 0.0
            for v in branches:
                if variant == "weighted_normalized":
                    x, y = emb[i][0][v], emb[j][0][v]
                    num += length[v] * abs(x - y)
                    den += length[v] * (x + y)
                else:
                    x, y = emb[i][1][v], emb[j][1][v]
                    num += length[v] * abs(x - y)
                    den += length[v] * max(x, y)
            out.append(num / den if den > 0 else 0.0)
    return out
