"""GRNG, pivot domains and the staged method's intermediates by definition.

Oracle; test infrastructure only.  Inputs are grid integers: point coordinates
``K`` (int64) and radii ``R`` (int64, same 2**-q units).  Every decision uses
exact integers: squared distances directly, and ``exact.sqrt_plus_lt`` where a
distance is offset by a radius.

Definitions followed:
* pivot domain D(p, r) = {x : d(x,p) <= r}             (Section 1, pivot domain equation)
* delta_max(p) = max over members x of d(x, p)           (Section 2, Proposition 3)
* GRNG link (i, j) iff no k with
      d(k,i) < d(i,j) - (2 r_i + r_j)  and  d(k,j) < d(i,j) - (r_i + 2 r_j)
                                                         (Section 2, Definition 1)
* virtual-pivot GRNG of a point x (x as a zero-radius pivot): pivot j is kept
  iff no k with d(x,k) < d(x,j) - r_j and d(j,k) < d(x,j) - 2 r_j
                                                         (Section 2, Proposition 1)
* relative domain: fine pivot p' belongs to coarse (p, r) iff d(p,p') <= r - r'
                                                         (Section 3, relative pivot domain)
* mu_bar_max(x) = max over RNG neighbours y of d(x,y);
  mu_max(p) = max over members x of [mu_bar_max(x) + d(x,p)]  (Section 2, Stage VII)
"""
from __future__ import annotations

import math

import numpy as np

from .exact import sqdist_rows, sqrt_plus_lt


def in_glune(d2_ki: int, d2_kj: int, d2_ij: int, ri: int, rj: int) -> bool:
    """k lies in the generalized lune of (i, r_i), (j, r_j) (Definition 1)."""
    return (sqrt_plus_lt(d2_ki, 2 * ri + rj, d2_ij)
            and sqrt_plus_lt(d2_kj, ri + 2 * rj, d2_ij))


def grng_edges(Kp: np.ndarray, R) -> np.ndarray:
    """Sorted (i < j) pairs of GRNG over pivot coordinates ``Kp`` with radii ``R`` (O(M^3))."""
    m = Kp.shape[0]
    D = sqdist_rows(Kp, np.arange(m))
    R = [int(r) for r in R]
    out = []
    for i in range(m):
        for j in range(i + 1, m):
            blocked = False
            for k in range(m):
                if k == i or k == j:
                    continue
                if in_glune(D[k, i], D[k, j], D[i, j], R[i], R[j]):
                    blocked = True
                    break
            if not blocked:
                out.append((i, j))
    return np.asarray(out, dtype=np.int64).reshape(-1, 2)


def membership(K: np.ndarray, pivot_ids, R) -> np.ndarray:
    """Boolean [n, m]: point x belongs to the domain of pivot p (d^2 <= r^2, exact)."""
    D = sqdist_rows(K, np.arange(K.shape[0]), np.asarray(pivot_ids))
    R = np.asarray(R, dtype=np.int64)
    return D <= (R * R)[None, :]


def delta_max_sq(K: np.ndarray, pivot_ids, R) -> np.ndarray:
    """Squared delta_max per pivot: the largest member squared distance (-1 if no member)."""
    D = sqdist_rows(K, np.arange(K.shape[0]), np.asarray(pivot_ids))
    M = membership(K, pivot_ids, R)
    return np.where(M, D, -1).max(axis=0)


def virtual_grng(K: np.ndarray, x: int, pivot_ids, R) -> np.ndarray:
    """Indices j (into pivot_ids) kept in the virtual-pivot GRNG of point x (Proposition 1)."""
    pid = np.asarray(pivot_ids)
    m = len(pid)
    dx = sqdist_rows(K, [x], pid)[0]
    Dp = sqdist_rows(K, pid, pid)
    keep = []
    for j in range(m):
        rj = int(R[j])
        blocked = any(
            sqrt_plus_lt(dx[k], rj, dx[j]) and sqrt_plus_lt(Dp[j, k], 2 * rj, dx[j])
            for k in range(m) if k != j)
        if not blocked:
            keep.append(j)
    return np.asarray(keep, dtype=np.int64)


def relative_membership(Kc: np.ndarray, Rc, Kf: np.ndarray, Rf) -> np.ndarray:
    """Boolean [mc, mf]: fine pivot f lies in the relative domain of coarse pivot c."""
    D = np.zeros((Kc.shape[0], Kf.shape[0]), dtype=np.int64)
    for t in range(Kc.shape[1]):
        diff = Kc[:, t][:, None] - Kf[:, t][None, :]
        D += diff * diff
    slack = np.asarray(Rc, dtype=np.int64)[:, None] - np.asarray(Rf, dtype=np.int64)[None, :]
    return (slack >= 0) & (D <= slack * slack)


def mu_bar_max_sq(n: int, K: np.ndarray, edges: np.ndarray) -> np.ndarray:
    """Squared mu_bar_max per point: largest squared length of its RNG edges (0 if none)."""
    out = np.zeros(n, dtype=np.int64)
    for u, v in np.asarray(edges).reshape(-1, 2):
        d2 = int(((K[u] - K[v]) ** 2).sum())
        out[u] = max(out[u], d2)
        out[v] = max(out[v], d2)
    return out


def mu_max(K: np.ndarray, pivot_ids, R, mu_bar_sq: np.ndarray) -> np.ndarray:
    """mu_max per pivot in grid units, as float64 (a sum of two square roots; diagnostic only)."""
    M = membership(K, pivot_ids, R)
    D = sqdist_rows(K, np.arange(K.shape[0]), np.asarray(pivot_ids))
    val = np.sqrt(mu_bar_sq.astype(np.float64))[:, None] + np.sqrt(D.astype(np.float64))
    return np.where(M, val, -math.inf).max(axis=0)
