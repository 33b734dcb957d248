"""Eulerian path over a built graph -- TEST INFRASTRUCTURE ONLY.

The assembly output of an A-Bruijn graph is an Eulerian path that uses every
edge as many times as its counter says (Background; Figure 1 caption).  For a
single error-free read whose walk is the only Eulerian path, the path spells
the read back, which pins the whole build: vertex keys, letter codes, edge
counts and the target rule together.

Hierholzer's algorithm (1873), iterative form, over edge multiplicities.
"""

from __future__ import annotations

import numpy as np

LETTERS = "ACTG"


def eulerian_spelling(keys, counts, k: int) -> str | None:
    """Spell one Eulerian path of the graph, or None if none exists.

    The walk starts at the vertex whose out-degree exceeds its in-degree by
    one (or at any vertex with an out-edge if the graph is balanced).
    """
    keys = [int(x) for x in np.asarray(keys, dtype=np.uint64)]
    counts = np.asarray(counts, dtype=np.int64).reshape(-1, 4)
    mask = (1 << (2 * (k - 1))) - 1
    index = {key: i for i, key in enumerate(keys)}
    remaining = counts.copy()
    indeg = np.zeros(len(keys), dtype=np.int64)
    for u in range(len(keys)):
        for c in range(4):
            if counts[u, c]:
                t = ((keys[u] << 2) | c) & mask
                if t not in index:
                    return None
                indeg[index[t]] += counts[u, c]
    outdeg = counts.sum(axis=1)
    diff = outdeg - indeg
    if np.any(diff > 1) or np.any(diff < -1) or (diff == 1).sum() > 1:
        return None
    if outdeg.sum() == 0:
        return None
    starts = np.nonzero(diff == 1)[0]
    start = int(starts[0]) if starts.size else int(np.nonzero(outdeg)[0][0])

    # iterative Hierholzer: stack of (vertex, letter that led here)
    stack = [(start, None)]
    path = []
    while stack:
        v, via = stack[-1]
        for c in range(4):
            if remaining[v, c]:
                remaining[v, c] -= 1
                t = index[((keys[v] << 2) | c) & mask]
                stack.append((t, c))
                break
        else:
            path.append(stack.pop())
    if remaining.sum():
        return None  # disconnected edges remain
    path.reverse()
    n = k - 1
    first = keys[path[0][0]]
    s = "".join(LETTERS[(first >> (2 * (n - 1 - i))) & 3] for i in range(n))
    return s + "".join(LETTERS[c] for _, c in path[1:])
