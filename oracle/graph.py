"""Graph neighbourhoods (oracle; test infrastructure only).

N_i is the set of senders j of edges j -> i (Sec. III-A): the incoming-edge
CSR row of i.  Tilde N_i = N_i U {i} (Sec. V-B proof).  With L message-passing
rounds, node i's next state depends on x^j for every j that reaches i in at
most L hops, so the Jacobian row i has a block for each such j.
"""
from __future__ import annotations

import numpy as np


def in_neighbours(row_ptr, col, i):
    """N_i: the senders of incoming edges of node i."""
    return [int(j) for j in col[row_ptr[i]:row_ptr[i + 1]]]


def ball(row_ptr, col, i, L):
    """Nodes that reach i in at most L hops along edges (breadth-first), sorted."""
    seen = {i}
    frontier = [i]
    for _ in range(L):
        nxt = []
        for n in frontier:
            for j in in_neighbours(row_ptr, col, n):
                if j not in seen:
                    seen.add(j)
                    nxt.append(j)
        frontier = nxt
    return sorted(seen)


def jacobian_pattern(row_ptr, col, M, L):
    """Block pattern of A_k: row i holds ball(i, L) in ascending order."""
    prow = np.zeros(M + 1, dtype=np.int32)
    pcol = []
    for i in range(M):
        b = ball(row_ptr, col, i, L)
        pcol.extend(b)
        prow[i + 1] = prow[i] + len(b)
    return prow, np.asarray(pcol, dtype=np.int32)
