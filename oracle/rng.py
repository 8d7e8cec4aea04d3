"""RNG, Gabriel graph and query rows by definition (oracle; test infrastructure only).

All functions take grid integers (see ``exact.to_grid``) and work on exact
int64 squared distances, so "<" below is the exact real comparison.

RNG (Section 1, the RNG definition equation): u and v are linked iff for every
other point z, max(d(z,u), d(z,v)) >= d(u,v).  Comparing squared distances is
the same decision since squaring is monotone on non-negative numbers.  Ties
(max == d) keep the edge: the lune is the open intersection of the two balls.

Gabriel graph (Section 1): u and v are linked iff for every other z,
d^2(z,u) + d^2(z,v) >= d^2(u,v).

Other metrics (the paper's setting is a general metric space, Section 1):
``rng_edges_metric`` applies the same RNG definition with the L1 (sum of
absolute differences) or L-infinity (largest absolute difference) distance,
again on exact integers.
"""
from __future__ import annotations

import numpy as np

from .exact import sqdist_rows


def _full_sqdist(K: np.ndarray) -> np.ndarray:
    return sqdist_rows(K, np.arange(K.shape[0]))


def rng_edges(K: np.ndarray) -> np.ndarray:
    """Sorted (u < v) int64 pairs of RNG(S): O(N^3) brute force over all witnesses."""
    n = K.shape[0]
    D = _full_sqdist(K)
    out = []
    for u in range(n - 1):
        du = D[u]                       # d^2(u, .)
        v = np.arange(u + 1, n)
        duv = du[v]                     # d^2(u, v) for each candidate v
        # witness[v, z]: z strictly inside lune(u, v).  z = u and z = v never
        # qualify (d(u,u) = 0 but d(v,u) = d(u,v) is not < d(u,v)).
        witness = (du[None, :] < duv[:, None]) & (D[v] < duv[:, None])
        alive = ~witness.any(axis=1)
        out.extend((u, int(w)) for w in v[alive])
    return np.asarray(out, dtype=np.int64).reshape(-1, 2)


def rng_edges_loops(K) -> list:
    """Third, loop-only implementation for tiny inputs (pure Python integers)."""
    pts = [tuple(int(c) for c in row) for row in np.asarray(K)]
    n = len(pts)

    def d2(a, b):
        return sum((x - y) ** 2 for x, y in zip(pts[a], pts[b]))

    edges = []
    for u in range(n):
        for v in range(u + 1, n):
            duv = d2(u, v)
            if all(max(d2(z, u), d2(z, v)) >= duv for z in range(n) if z != u and z != v):
                edges.append((u, v))
    return edges


def gabriel_edges(K: np.ndarray) -> np.ndarray:
    """Sorted (u < v) pairs of the Gabriel graph by definition."""
    n = K.shape[0]
    D = _full_sqdist(K)
    out = []
    for u in range(n - 1):
        v = np.arange(u + 1, n)
        duv = D[u, v]
        inside = (D[u][None, :] + D[v] < duv[:, None])
        inside[np.arange(len(v)), v] = False
        inside[:, u] = False
        alive = ~inside.any(axis=1)
        out.extend((u, int(w)) for w in v[alive])
    return np.asarray(out, dtype=np.int64).reshape(-1, 2)


def query_row(K: np.ndarray, qk) -> np.ndarray:
    """RNG neighbours of an external query point within S u {Q} (the output of Algorithm 1).

    x in S is a neighbour iff no z in S \\ {x} has max(d(Q,z), d(x,z)) < d(Q,x).
    """
    qk = np.asarray(qk, dtype=np.int64).reshape(1, -1)
    dq = sqdist_rows(np.vstack([qk, K]), [0])[0, 1:]      # d^2(Q, x)
    D = _full_sqdist(K)
    witness = (dq[None, :] < dq[:, None]) & (D < dq[:, None])
    np.fill_diagonal(witness, False)
    return np.nonzero(~witness.any(axis=1))[0].astype(np.int64)


def nearest_neighbour(K: np.ndarray) -> np.ndarray:
    """Index of the nearest other point of each point (ties: smallest index)."""
    D = _full_sqdist(K).astype(np.float64)
    np.fill_diagonal(D, np.inf)
    return D.argmin(axis=1)


def average_degree(num_edges: int, n: int) -> float:
    """Average degree of an undirected graph: each edge adds one to two degrees."""
    return 2.0 * num_edges / n


def metric_dists(K: np.ndarray, metric: str) -> np.ndarray:
    """All pairwise distances of integer points, exact: 'l1' = sum of |differences|,
    'linf' = largest |difference|, 'l2sq' = squared Euclidean distance."""
    K = np.asarray(K, dtype=np.int64)
    n = K.shape[0]
    out = np.zeros((n, n), dtype=np.int64)
    for t in range(K.shape[1]):
        diff = np.abs(K[:, t][:, None] - K[:, t][None, :])
        if metric == "l1":
            out += diff
        elif metric == "linf":
            out = np.maximum(out, diff)
        elif metric == "l2sq":
            out += diff * diff
        else:
            raise ValueError(metric)
    return out


def rng_edges_metric(K: np.ndarray, metric: str) -> np.ndarray:
    """RNG under another metric: (u, v) linked iff no z has max(d(u,z), d(v,z)) < d(u,v)."""
    n = K.shape[0]
    D = metric_dists(K, metric)
    out = []
    for u in range(n - 1):
        v = np.arange(u + 1, n)
        duv = D[u, v]
        witness = (D[u][None, :] < duv[:, None]) & (D[v] < duv[:, None])
        alive = ~witness.any(axis=1)
        out.extend((u, int(w)) for w in v[alive])
    return np.asarray(out, dtype=np.int64).reshape(-1, 2)


def rng_edges_metric_loops(K, metric: str) -> list:
    """Loop-only version of rng_edges_metric for tiny inputs (Python integers)."""
    pts = [tuple(int(c) for c in row) for row in np.asarray(K)]
    n = len(pts)

    def dist(a, b):
        diffs = [abs(x - y) for x, y in zip(pts[a], pts[b])]
        return sum(diffs) if metric == "l1" else max(diffs, default=0)

    return [(u, v) for u in range(n) for v in range(u + 1, n)
            if all(max(dist(z, u), dist(z, v)) >= dist(u, v) for z in range(n) if z != u and z != v)]
