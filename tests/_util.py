"""Small helpers shared by the tests (input construction only)."""
import numpy as np

import synth


def tree(parent, length):
    parent = np.asarray(parent, dtype=np.int64)
    length = np.asarray(length, dtype=np.float64)
    has_child = np.zeros(parent.shape[0], bool)
    has_child[parent[parent >= 0]] = True
    return synth.Tree(parent=parent, length=length, n_tips=int((~has_child).sum()))


def table(rows):
    """rows: list of {tip node id: count}."""
    indptr = [0]
    tips, counts = [], []
    for r in rows:
        for t in sorted(r):
            tips.append(int(t))
            counts.append(int(r[t]))
        indptr.append(len(tips))
    return synth.Table(indptr=np.asarray(indptr, np.int64), tips=np.asarray(tips, np.int64),
                       counts=np.asarray(counts, np.int64))


def squareform(cond, n):
    d = np.zeros((n, n))
    k = 0
    for i in range(n):
        for j in range(i + 1, n):
            d[i, j] = d[j, i] = cond[k]
            k += 1
    return d


def tip_ids(t):
    has_child = np.zeros(t.parent.shape[0], bool)
    has_child[t.parent[t.parent >= 0]] = True
    return np.nonzero(~has_child)[0]


def random_rows(rng, tips, n_samples, max_nnz=None, zero_prob=0.0):
    """Random samples on the given tips, each with a nonzero total."""
    tips = np.asarray(tips)
    rows = []
    for _ in range(n_samples):
        k = int(rng.integers(1, (max_nnz or tips.shape[0]) + 1))
        k = min(k, tips.shape[0])
        pick = rng.choice(tips, size=k, replace=False)
        r = {int(t): int(rng.integers(1, 20)) for t in pick}
        if zero_prob and len(r) > 1:
            for t in list(r)[1:]:
                if rng.random() < zero_prob:
                    r[t] = 0
        rows.append(r)
    return rows
