"""RNG, Gabriel graph and query rows by definition (oracle; test infrastructure only).

All functions take grid integers (see ``exact.to_grid``) and work on exact
int64 squared distances, so "<" below is the exact real comparison.

RNG (Section 1, the RNG definition equation): u and v are linked iff for every
other point z, max(d(z,u), d(z,v)) >= d(u,v).  Comparing squared distances is
the same decision since squaring is monotone on non-negative numbers.  Ties
(max == d) keep the edge: the lune is the open intersection of the two balls.

Gabriel graph (Section 1): u and v are linked iff for every other z,
d^2(z,u) + d^2(z,v) >= d^2(u,v).

Lune-based beta-skeleton (named in Section 1 among the proximity graphs; the
paper gives no formula, so this is the standard lune-based form of the work it
cites, for beta >= 1): u and v are linked iff no other z lies in both open
balls of radius beta d(u,v)/2 centred at (1 - beta/2) u + (beta/2) v and
(beta/2) u + (1 - beta/2) v.  beta = 1 gives the Gabriel graph, beta = 2 the
RNG.  With beta = a/4 both balls' tests become integer comparisons after
multiplying by 16: |8(z - u) + a(u - v)|^2 < a^2 d^2(u,v) and
|8(z - v) + a(v - u)|^2 < a^2 d^2(u,v).

Other metrics (the paper's setting is a general metric space, Section 1):
``rng_edges_metric`` applies the same RNG definition with the L1 (sum of
absolute differences) or L-infinity (largest absolute difference) distance,
again on exact integers.
"""
from __future__ import annotations

from fractions import Fraction

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


def _beta_checked(K: np.ndarray, beta_quarters: int):
    a = int(beta_quarters)
    if a < 4:
        raise ValueError("the lune-based beta-skeleton needs beta >= 1")
    K = np.asarray(K, dtype=np.int64)
    n, d = K.shape
    span = int((K.max(axis=0) - K.min(axis=0)).max()) if n else 0
    if d * ((8 + a) * span) ** 2 >= 2 ** 62 or a * a * d * span * span >= 2 ** 62:
        raise ValueError("coordinates too large for the int64 beta-skeleton oracle")
    return K, a


def _beta_alive(K: np.ndarray, u: int, v: np.ndarray, a: int) -> np.ndarray:
    """alive[k]: no point other than u and v[k] lies in the beta-lune of (u, v[k])."""
    uv = K[u][None, :] - K[v]                                    # u - v, (|v|, d)
    rhs = a * a * (uv * uv).sum(axis=1)                          # a^2 d^2(u, v)
    e1 = 8 * (K[None, :, :] - K[u][None, None, :]) + a * uv[:, None, :]   # 8(z - u) + a(u - v)
    e2 = 8 * (K[None, :, :] - K[v][:, None, :]) - a * uv[:, None, :]      # 8(z - v) + a(v - u)
    inside = ((e1 * e1).sum(axis=2) < rhs[:, None]) & ((e2 * e2).sum(axis=2) < rhs[:, None])
    inside[:, u] = False
    inside[np.arange(len(v)), v] = False
    return ~inside.any(axis=1)


def beta_skeleton_edges(K: np.ndarray, beta_quarters: int) -> np.ndarray:
    """Sorted (u < v) pairs of the lune-based beta-skeleton, beta = beta_quarters / 4 >= 1,
    on exact int64 arithmetic (raises where int64 could overflow)."""
    K, a = _beta_checked(K, beta_quarters)
    n = K.shape[0]
    out = []
    for u in range(n - 1):
        v = np.arange(u + 1, n)
        out.extend((u, int(w)) for w in v[_beta_alive(K, u, v, a)])
    return np.asarray(out, dtype=np.int64).reshape(-1, 2)


def beta_skeleton_row(K: np.ndarray, i: int, beta_quarters: int) -> np.ndarray:
    """Sorted neighbours of point i in the beta-skeleton of K (the test is
    symmetric in the pair's two points)."""
    K, a = _beta_checked(K, beta_quarters)
    v = np.array([w for w in range(K.shape[0]) if w != i], dtype=np.int64)
    return v[_beta_alive(K, i, v, a)]


def beta_skeleton_edges_loops(K, beta: Fraction) -> list:
    """Loop-only beta-skeleton for tiny inputs, in exact rationals: the two
    centres are formed as points and the squared radius as (beta d / 2)^2."""
    pts = [tuple(Fraction(int(c)) for c in row) for row in np.asarray(K)]
    n = len(pts)
    beta = Fraction(beta)

    def d2(p, q):
        return sum((x - y) ** 2 for x, y in zip(p, q))

    edges = []
    for u in range(n):
        for v in range(u + 1, n):
            pu, pv = pts[u], pts[v]
            c1 = tuple((1 - beta / 2) * x + beta / 2 * y for x, y in zip(pu, pv))
            c2 = tuple(beta / 2 * x + (1 - beta / 2) * y for x, y in zip(pu, pv))
            r2 = (beta / 2) ** 2 * d2(pu, pv)
            if all(not (d2(pts[z], c1) < r2 and d2(pts[z], c2) < r2) for z in range(n) if z != u and z != v):
                edges.append((u, v))
    return edges
