"""Exact arithmetic on grid inputs (oracle; test infrastructure only).

A coordinate x is on the 2**-q grid when x * 2**q is an integer.  For such
inputs the squared Euclidean distance is an integer number of 2**-2q units;
this module computes that integer exactly and decides comparisons between
distances exactly.  Decisions that involve a distance minus a radius (the
generalized lune of Definition 1, Section 2, and the virtual pivot tests of
Propositions 1-2) are square-root comparisons; ``sqrt_plus_lt`` decides them
exactly with integers.
"""
from __future__ import annotations

import math
from decimal import Decimal, getcontext

import numpy as np


GRID_KMAX = 2 ** 24          # every grid integer satisfies |k| < 2**24
GRID_SUM_LIMIT = 2 ** 51     # and dimension * kmax**2 < 2**51


def to_grid(X, q: int) -> np.ndarray:
    """Exact integer coordinates k = x * 2**q (int64); raises if x is off the grid.

    Enforces the exactness contract the oracle relies on: |k| < 2**24 and
    d * kmax**2 < 2**51, so a squared distance, (2 kmax)**2 * d < 2**53, and
    every partial sum of one fit int64 (and float64) with room to spare.
    """
    A = np.asarray(X, dtype=np.float64) * (2.0 ** q)
    K = np.rint(A)
    if not np.array_equal(A, K):
        raise ValueError(f"input is not on the 2**-{q} grid")
    if K.size:
        kmax = int(np.abs(K).max())
        if kmax >= GRID_KMAX:
            raise ValueError("grid integers must satisfy |k| < 2**24")
        d = K.shape[-1] if K.ndim > 1 else 1
        if d * kmax * kmax >= GRID_SUM_LIMIT:
            raise ValueError("grid integers too large: need d * kmax**2 < 2**51")
    return K.astype(np.int64)


def radius_to_grid(r, q: int) -> np.ndarray:
    """Radii as exact grid integers (int64); radii must be >= 0 and on the grid."""
    R = to_grid(np.asarray(r, dtype=np.float64).reshape(-1, 1), q).reshape(-1)
    if np.any(R < 0):
        raise ValueError("negative radius")
    return R


def sqdist_rows(K: np.ndarray, rows, cols=None) -> np.ndarray:
    """Exact squared distances (int64 grid units) between K[rows] and K[cols].

    Plain definition: sum over coordinates of the squared integer difference.
    """
    A = K[np.asarray(rows)]
    B = K if cols is None else K[np.asarray(cols)]
    out = np.zeros((A.shape[0], B.shape[0]), dtype=np.int64)
    for t in range(K.shape[1]):
        diff = A[:, t][:, None] - B[:, t][None, :]
        out += diff * diff
    return out


def sqdist_py(a, b) -> int:
    """Squared distance of two integer points with Python integers (no overflow possible)."""
    return sum((int(u) - int(v)) ** 2 for u, v in zip(a, b))


def sqrt_plus_lt(a: int, c: int, b: int) -> bool:
    """Exact truth of  sqrt(a) + c < sqrt(b)  for integers a, b >= 0 and c >= 0.

    sqrt(a) < sqrt(b) - c needs sqrt(b) > c, i.e. c*c < b; squaring both
    (non-negative) sides then gives a < b - 2c*sqrt(b) + c*c, i.e.
    2c*sqrt(b) < T with T = b + c*c - a, which needs T > 0 and, squared again,
    4*c*c*b < T*T.  With c = 0 it reduces to a < b.
    """
    a, b, c = int(a), int(b), int(c)
    if c < 0 or a < 0 or b < 0:
        raise ValueError("sqrt_plus_lt needs non-negative arguments")
    if c * c >= b:
        return False
    t = b + c * c - a
    return t > 0 and 4 * c * c * b < t * t


def sqrt_plus_lt_decimal(a: int, c: int, b: int, digits: int = 120) -> bool:
    """Independent check of ``sqrt_plus_lt`` with high-precision decimal square roots."""
    getcontext().prec = digits
    lhs = Decimal(int(a)).sqrt() + Decimal(int(c))
    rhs = Decimal(int(b)).sqrt()
    return lhs < rhs


def isqrt_floor(v: int) -> int:
    return math.isqrt(int(v))
