"""Seeded synthetic workloads for the exact RNG / GRNG build.

This module only draws inputs: point sets, pivot layers (pivot ids and ball
radii) and insertion batches.  It holds none of the method's arithmetic (no
lune test, no G-lune test, no pruning); both the oracle and the HIP library
consume what it produces, and neither is imported here.

Every coordinate is put on a dyadic grid: it is k * 2**-q for an integer k with
|k| < 2**24, so the float32 value is exact and the squared distance of two
points is an integer multiple of 2**-2q that float64 holds exactly.  Radii are
on the same grid and rounded up, so a pivot ball always holds the points the
radius rule meant it to hold.

Workloads (the paper's experiments use uniform and clustered synthetic data,
Section 4; the shapes below are the build targets):

* ``uniform2d``      N points i.i.d. uniform in [0,1)^2, no pivots.
* ``clustered``      Gaussian mixture of equally weighted isotropic clusters,
                     centres uniform in [0,10]^D, with M random pivots whose
                     radius is the distance to the k-th nearest other point.
* ``subspace3``      points on a random 8-dimensional linear subspace of R^32
                     plus isotropic noise, with a nested two-level pivot layer
                     (coarse pivots are a subset of the fine pivots).
* ``insert_batches`` batch sizes drawn log-uniform, fresh points from the same
                     mixture as ``clustered``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ROOT_SEED = 2208_10022
# One child stream per workload family; spawn keys are fixed so that adding a
# family never changes the inputs of another.
_FAMILY = {"uniform2d": 0, "clustered": 1, "subspace3": 2, "insert": 3, "mlp": 4, "subspace_layers": 5}


def _stream(family: str, *sub: int) -> np.random.Generator:
    ss = np.random.SeedSequence(ROOT_SEED, spawn_key=(_FAMILY[family],) + tuple(sub))
    return np.random.Generator(np.random.PCG64(ss))


@dataclass
class PivotLayer:
    pivot_ids: np.ndarray  # int32 [m], indices into the point set
    radii: np.ndarray      # float32 [m], on the grid, rounded up


@dataclass
class Workload:
    name: str
    X: np.ndarray                 # float32 [n, d], on the grid
    q: int                        # grid exponent: coordinates are k * 2**-q
    layers: list = field(default_factory=list)   # PivotLayer, coarsest first
    batches: list = field(default_factory=list)  # float32 [nb, d] each
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.X.shape[0])

    @property
    def d(self) -> int:
        return int(self.X.shape[1])


def quantize(x: np.ndarray, q: int) -> np.ndarray:
    """Round to the nearest multiple of 2**-q and return exact float32 values."""
    k = np.rint(np.asarray(x, dtype=np.float64) * (2.0 ** q))
    lim = 2.0 ** 24 - 1
    if np.any(np.abs(k) > lim):
        raise ValueError("coordinate magnitude exceeds the 24-bit grid at q=%d" % q)
    return (k * (2.0 ** -q)).astype(np.float32)


def grid_ints(X: np.ndarray, q: int) -> np.ndarray:
    """Integer grid coordinates k = x * 2**q as int64 (exact for grid input)."""
    k = np.asarray(X, dtype=np.float64) * (2.0 ** q)
    ki = np.rint(k)
    if not np.array_equal(k, ki):
        raise ValueError("input is not on the 2**-%d grid" % q)
    return ki.astype(np.int64)


def _sq_dists_to(Xi: np.ndarray, rows: np.ndarray) -> np.ndarray:
    """Exact squared distances (integer grid units) from points ``rows`` to all points.

    Input recipe helper for the k-NN radius rule.  Integer coordinates are
    below 2**24 and the dimension is small, so float64 holds every product and
    partial sum exactly and the matrix product is exact in any order.
    """
    Xf = Xi.astype(np.float64)
    if Xf.shape[1] * float(np.abs(Xf).max() if Xf.size else 0.0) ** 2 * 4 >= 2.0 ** 53:
        raise ValueError("grid too fine for exact float64 radius computation")
    R = Xf[rows]
    nx = np.einsum("ij,ij->i", Xf, Xf)
    nr = np.einsum("ij,ij->i", R, R)
    return nr[:, None] + nx[None, :] - 2.0 * (R @ Xf.T)


def _isqrt_ceil(v: int) -> int:
    s = math.isqrt(v)
    return s if s * s == v else s + 1


def knn_radii(X: np.ndarray, q: int, pivot_ids: np.ndarray, k: int, chunk: int = 256) -> np.ndarray:
    """Radius of each pivot = distance to its k-th nearest *other* point, rounded up to the grid."""
    Xi = grid_ints(X, q)
    out = np.empty(len(pivot_ids), dtype=np.float32)
    for s in range(0, len(pivot_ids), chunk):
        rows = np.asarray(pivot_ids[s:s + chunk], dtype=np.int64)
        D2 = _sq_dists_to(Xi, rows)
        D2[np.arange(len(rows)), rows] = np.inf  # exclude the pivot itself
        kth = np.partition(D2, k - 1, axis=1)[:, k - 1]
        for t, v in enumerate(kth):
            r_int = _isqrt_ceil(int(v))
            out[s + t] = np.float32(r_int * 2.0 ** -q)
    return out


def uniform2d(n: int = 1000, d: int = 2, sub: int = 0) -> Workload:
    """N points i.i.d. uniform in [0,1)^d, exact float32 multiples of 2**-24."""
    g = _stream("uniform2d", n, d, sub)
    q = 24
    k = g.integers(0, 2 ** 24, size=(n, d), dtype=np.int64)
    X = (k.astype(np.float64) * 2.0 ** -q).astype(np.float32)
    return Workload(name=f"uniform{d}d_n{n}", X=X, q=q)


def mixture_points(g: np.random.Generator, centres: np.ndarray, n: int, sigma: float, q: int) -> np.ndarray:
    lab = g.integers(0, centres.shape[0], size=n)
    X = centres[lab] + sigma * g.standard_normal((n, centres.shape[1]))
    return quantize(X, q)


def clustered(n: int = 100_000, d: int = 16, clusters: int = 32, sigma: float = 0.5,
              m: int = 1000, knn: int = 100, q: int = 19, sub: int = 0) -> Workload:
    """Gaussian mixture with one random pivot layer (two-layer GRNG -> RNG workload)."""
    g = _stream("clustered", n, d, clusters, m, sub)
    centres = g.uniform(0.0, 10.0, size=(clusters, d))
    X = mixture_points(g, centres, n, sigma, q)
    layers = []
    if m > 0:
        pid = np.sort(g.choice(n, size=m, replace=False)).astype(np.int32)
        rad = knn_radii(X, q, pid, min(knn, n - 1))
        layers.append(PivotLayer(pid, rad))
    return Workload(name=f"clustered_n{n}_d{d}_c{clusters}_m{m}", X=X, q=q, layers=layers,
                    meta={"centres": centres, "sigma": sigma, "knn": knn})


def insert_batches(base: Workload, n_batches: int = 64, lo: int = 1000, hi: int = 50_000,
                   sub: int = 0) -> list:
    """Batches for incremental insertion: sizes log-uniform in [lo, hi], same mixture as ``base``."""
    g = _stream("insert", base.n, base.d, n_batches, lo, hi, sub)
    sizes = np.rint(np.exp(g.uniform(math.log(lo), math.log(hi), size=n_batches))).astype(np.int64)
    centres = base.meta["centres"]
    sigma = base.meta["sigma"]
    return [mixture_points(g, centres, int(s), sigma, base.q) for s in sizes]


def subspace3(n: int = 1_000_000, d: int = 32, latent: int = 8, noise: float = 0.01,
              m_fine: int = 3000, m_coarse: int = 100, q: int = 21, sub: int = 0) -> Workload:
    """Points on a random ``latent``-dim subspace of R^d plus noise, with nested pivot layers.

    Fine radius: distance to the ceil(n/m_fine)-th nearest other point.  Coarse
    radius: the ceil(m_fine/m_coarse)-th smallest of d(p, fine p') + r(fine p')
    over fine pivots p', so every coarse ball wholly holds at least that many
    fine balls.  Coarse pivots are drawn from the fine pivots (nested layers).
    """
    g = _stream("subspace3", n, d, latent, m_fine, m_coarse, sub)
    B, _ = np.linalg.qr(g.standard_normal((d, latent)))
    U = g.uniform(0.0, 1.0, size=(n, latent))
    X = quantize(U @ B.T + noise * g.standard_normal((n, d)), q)
    fine = np.sort(g.choice(n, size=m_fine, replace=False)).astype(np.int32)
    kf = min(-(-n // m_fine), n - 1)
    r_fine = knn_radii(X, q, fine, kf)
    coarse = np.sort(g.choice(fine, size=m_coarse, replace=False)).astype(np.int32)
    Xi = grid_ints(X, q)
    D2 = _sq_dists_to(Xi[fine], np.searchsorted(fine, coarse))  # coarse x fine, exact
    rf_int = np.rint(r_fine.astype(np.float64) * 2.0 ** q).astype(np.int64)
    kc = min(-(-m_fine // m_coarse), m_fine)
    r_coarse = np.empty(m_coarse, dtype=np.float32)
    for i in range(m_coarse):
        tot = np.array([_isqrt_ceil(int(v)) for v in D2[i]], dtype=np.int64) + rf_int
        r_coarse[i] = np.float32(int(np.partition(tot, kc - 1)[kc - 1]) * 2.0 ** -q)
    layers = [PivotLayer(coarse, r_coarse), PivotLayer(fine, r_fine)]
    return Workload(name=f"subspace_n{n}_d{d}_m{m_coarse}-{m_fine}", X=X, q=q, layers=layers)


def subspace_layers(n: int, d: int = 32, latent: int = 8, noise: float = 0.01, ms=(30, 300, 3000),
                    q: int = 21, sub: int = 0) -> Workload:
    """The subspace law of ``subspace3`` with any number of nested pivot layers.

    ``ms`` lists the layer sizes coarsest first.  The finest layer is drawn
    from the points, each coarser layer from the next finer one.  Radii: the
    finest layer's is the distance to the ceil(n/M)-th nearest other point;
    a coarser layer's the ceil(M_finer/M)-th smallest of d(p, p') + r(p')
    over the next finer layer's pivots p' (so its ball wholly holds that many
    finer balls).  The points depend on (n, d, latent, sub) only, so
    hierarchies of the same points can be compared; a separate seed stream
    from ``subspace3``.
    """
    ms = [int(m) for m in ms]
    assert all(a < b for a, b in zip(ms, ms[1:])) and ms[-1] <= n
    g = _stream("subspace_layers", n, d, latent, sub)   # the points do not depend on the layers
    B, _ = np.linalg.qr(g.standard_normal((d, latent)))
    U = g.uniform(0.0, 1.0, size=(n, latent))
    X = quantize(U @ B.T + noise * g.standard_normal((n, d)), q)
    Xi = grid_ints(X, q)
    g = _stream("subspace_layers", n, d, latent, sub, *ms)
    fine = np.sort(g.choice(n, size=ms[-1], replace=False)).astype(np.int32)
    r_fine = knn_radii(X, q, fine, min(-(-n // ms[-1]), n - 1))
    layers = [PivotLayer(fine, r_fine)]
    for m in reversed(ms[:-1]):
        finer = layers[0]
        ids = np.sort(g.choice(finer.pivot_ids, size=m, replace=False)).astype(np.int32)
        D2 = _sq_dists_to(Xi[finer.pivot_ids], np.searchsorted(finer.pivot_ids, ids))
        rf = np.rint(finer.radii.astype(np.float64) * 2.0 ** q).astype(np.int64)
        k = min(-(-len(finer.pivot_ids) // m), len(finer.pivot_ids))
        rad = np.empty(m, dtype=np.float32)
        for i in range(m):
            tot = np.array([_isqrt_ceil(int(v)) for v in D2[i]], dtype=np.int64) + rf
            rad[i] = np.float32(int(np.partition(tot, k - 1)[k - 1]) * 2.0 ** -q)
        layers.insert(0, PivotLayer(ids, rad))
    return Workload(name="subspace_n%d_d%d_m%s" % (n, d, "-".join(map(str, ms))), X=X, q=q, layers=layers)


def queries_like(base: Workload, nq: int, sub: int = 0) -> np.ndarray:
    """Fresh query points from the same mixture as a ``clustered`` workload."""
    g = _stream("clustered", base.n, base.d, 7919, nq, sub)
    return mixture_points(g, base.meta["centres"], nq, base.meta["sigma"], base.q)
