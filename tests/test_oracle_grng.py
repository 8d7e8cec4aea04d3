"""Pins of the GRNG / domain oracle and of the C oracle (CPU only).

The GRNG oracle is pinned by the paper's own statements about the graph
(Section 2, after Definition 1): GRNG = RNG when every radius is 0, GRNG is a
superset of RNG, it is connected, it grows with the radii and is complete once
the radius exceeds a sixth of the largest distance (GRNG examples figure).  The
paper's pruning theorems (Theorem 1, Propositions 1 and 3, Theorem 2) are
checked as implications between the GRNG, domain and RNG oracles on random
small hierarchies: a pruned pair must never be an exact RNG edge.
"""
import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components

import synth
from oracle import exact, grng, rng


def edge_set(E):
    return {(int(u), int(v)) for u, v in np.asarray(E).reshape(-1, 2)}


def test_sqrt_plus_lt_against_high_precision():
    g = np.random.default_rng(9)
    cases = []
    for _ in range(3000):
        s = int(g.integers(0, 2 ** 26))
        c = int(g.integers(0, 2 ** 24))
        a = s * s
        b = (s + c) ** 2                      # exact equality: sqrt(a) + c == sqrt(b)
        cases += [(a, c, b), (a, c, b + 1), (a, c, b - 1), (a + 1, c, b), (max(a - 1, 0), c, b)]
        cases.append((int(g.integers(0, 2 ** 52)), int(g.integers(0, 2 ** 25)), int(g.integers(0, 2 ** 52))))
    cases += [(0, 0, 0), (0, 0, 1), (1, 0, 1), (0, 1, 1), (0, 1, 2), (3, 0, 4)]
    for a, c, b in cases:
        want = exact.sqrt_plus_lt_decimal(a, c, b)
        assert exact.sqrt_plus_lt(a, c, b) == want, (a, c, b)


def test_c_predicate_matches_python(oracle_native):
    g = np.random.default_rng(10)
    for _ in range(20000):
        s = int(g.integers(0, 2 ** 26)); c = int(g.integers(0, 2 ** 25))
        b = (s + c) ** 2 + int(g.integers(-2, 3))
        a = s * s + int(g.integers(-2, 3))
        a, b = max(a, 0), max(b, 0)
        if a >= 2 ** 53 or b >= 2 ** 53:
            continue
        assert oracle_native.sqrt_plus_lt(a, c, b) == exact.sqrt_plus_lt(a, c, b)


def _rand_layer(g, m, d, hi, rmax):
    K = g.integers(0, hi, size=(m, d)).astype(np.int64)
    R = g.integers(0, rmax + 1, size=m).astype(np.int64)
    return K, R


def test_zero_radius_grng_is_the_rng():
    g = np.random.default_rng(12)
    for _ in range(10):
        K, _ = _rand_layer(g, 25, 2, 200, 0)
        assert edge_set(grng.grng_edges(K, np.zeros(len(K), np.int64))) == edge_set(rng.rng_edges(K))


def test_grng_superset_connected_and_monotone_in_radius():
    g = np.random.default_rng(13)
    for _ in range(8):
        K, R = _rand_layer(g, 30, 2, 1000, 40)
        E0 = edge_set(rng.rng_edges(K))
        E1 = edge_set(grng.grng_edges(K, R))
        E2 = edge_set(grng.grng_edges(K, R * 2 + 3))
        assert E0 <= E1 <= E2
        A = np.zeros((len(K), len(K)))
        for u, v in E1:
            A[u, v] = A[v, u] = 1
        assert connected_components(csr_matrix(A))[0] == 1


def test_grng_complete_once_radius_exceeds_a_sixth_of_the_diameter():
    pts = np.array([[int(v) for v in ln.split()] for ln in
                    open(__file__.replace("test_oracle_grng.py", "golden/grng_complete_threshold.txt"))
                    if ln.strip() and not ln.startswith("#")], dtype=np.int64)
    D = exact.sqdist_rows(pts, np.arange(len(pts)))
    dmax = float(np.sqrt(D.max()))
    r = int(np.ceil(dmax / 6.0))
    m = len(pts)
    assert len(edge_set(grng.grng_edges(pts, np.full(m, r)))) == m * (m - 1) // 2
    # below the threshold, the collinear triple (0,0),(10,0),(20,0) is not complete at r = 0
    assert (0, 2) not in edge_set(grng.grng_edges(pts, np.zeros(m, np.int64)))


def test_c_oracle_matches_python_grng(oracle_native):
    g = np.random.default_rng(14)
    for trial in range(6):
        m = 35
        K, R = _rand_layer(g, m, 3, 500 if trial % 2 else 60, 30)
        X = K.astype(np.float32)
        want = edge_set(grng.grng_edges(K, R))
        got = edge_set(oracle_native.grng_edges(X, R.astype(np.float32), 0))
        assert got == want


def test_c_oracle_matches_python_rng(oracle_native):
    g = np.random.default_rng(15)
    for d, n, hi in [(2, 300, 2 ** 20), (3, 250, 16), (7, 200, 1000), (1, 50, 30)]:
        K = g.integers(0, hi, size=(n, d)).astype(np.int64)
        X = K.astype(np.float32)
        want = edge_set(rng.rng_edges(K))
        assert edge_set(oracle_native.rng_edges(X, 0, threads=4)) == want
        for x in (0, n // 2, n - 1):
            row = {v for e in want for v in e if x in e and v != x} | {x for e in want if e == (x, x)}
            assert set(oracle_native.rng_row(X, 0, x).tolist()) == row
        rows = oracle_native.rng_rows(X, 0, [1, 2, 3], threads=3)
        assert [set(r.tolist()) for r in rows] == [set(oracle_native.rng_row(X, 0, x).tolist()) for x in (1, 2, 3)]
        Q = g.integers(0, hi, size=d).astype(np.int64)
        assert set(oracle_native.query_row(X, 0, Q.astype(np.float32)).tolist()) == set(rng.query_row(K, Q).tolist())


def test_c_oracle_on_grid_workload(oracle_native):
    W = synth.clustered(n=600, d=16, clusters=4, m=12, knn=20)
    K = exact.to_grid(W.X, W.q)
    assert edge_set(oracle_native.rng_edges(W.X, W.q)) == edge_set(rng.rng_edges(K))
    L = W.layers[0]
    R = exact.radius_to_grid(L.radii, W.q)
    assert edge_set(oracle_native.grng_edges(W.X[L.pivot_ids], L.radii, W.q)) == \
        edge_set(grng.grng_edges(K[L.pivot_ids], R))


# ---------------------------------------------------------------------------
# The paper's pruning theorems, as implications between the oracles.

def _hierarchy(seed, n=80, m=16, d=2):
    g = np.random.default_rng(seed)
    K = g.integers(0, 400, size=(n, d)).astype(np.int64)
    pid = np.sort(g.choice(n, size=m, replace=False))
    R = g.integers(5, 40, size=m).astype(np.int64)
    return K, pid, R


@pytest.mark.parametrize("seed", range(6))
def test_theorem1_and_propositions_never_prune_an_rng_edge(seed):
    K, pid, R = _hierarchy(seed)
    E = edge_set(rng.rng_edges(K))
    memb = grng.membership(K, pid, R)                  # [n, m]
    G = edge_set(grng.grng_edges(K[pid], R))
    n = len(K)
    vg = [set(grng.virtual_grng(K, x, pid, R).tolist()) for x in range(n)]
    # non-vacuous: the theorems do prune some pairs of this hierarchy
    pruned = sum(1 for u in range(n) for v in range(u + 1, n)
                 if not (set(np.nonzero(memb[v])[0].tolist()) <= vg[u]))
    assert pruned > 0 and len(G) < len(pid) * (len(pid) - 1) // 2
    for u, v in E:
        pu, pv = np.nonzero(memb[u])[0], np.nonzero(memb[v])[0]
        # Theorem 1: members of two unlinked pivot domains are never linked.
        for i in pu:
            for j in pv:
                if i != j:
                    assert (min(i, j), max(i, j)) in G
        # Propositions 1-2: all parents of v are in GRNG(u) and vice versa.
        assert set(pv.tolist()) <= vg[u] and set(pu.tolist()) <= vg[v]
    # Parents of a point always survive its own virtual-pivot test.
    for x in range(n):
        assert set(np.nonzero(memb[x])[0].tolist()) <= vg[x]


@pytest.mark.parametrize("seed", range(4))
def test_proposition3_domain_skip_never_drops_a_witness(seed):
    # A domain whose every member is outside lune(x, y) by the delta_max bound
    # holds no witness of (x, y): checked against exact witness sets.
    K, pid, R = _hierarchy(100 + seed)
    n = len(K)
    D = exact.sqdist_rows(K, np.arange(n))
    memb = grng.membership(K, pid, R)
    dmax = np.sqrt(np.maximum(grng.delta_max_sq(K, pid, R), 0).astype(float))
    skips = 0
    for x in range(0, n, 3):
        for y in range(x + 1, n, 2):
            dxy = np.sqrt(float(D[x, y]))
            for k, p in enumerate(pid):
                if not memb[:, k].any():
                    continue
                skip = max(np.sqrt(float(D[x, p])), np.sqrt(float(D[y, p]))) - dmax[k] >= dxy + 1e-9
                if skip:
                    skips += 1
                    members = np.nonzero(memb[:, k])[0]
                    w = (D[x, members] < D[x, y]) & (D[y, members] < D[x, y])
                    assert not w.any()
    assert skips > 0


def test_theorem2_coarse_nonlink_implies_fine_nonlink():
    g = np.random.default_rng(21)
    checks = 0
    for _ in range(5):
        Kf = g.integers(0, 600, size=(40, 2)).astype(np.int64)
        Rf = g.integers(0, 15, size=40).astype(np.int64)
        cidx = np.sort(g.choice(40, size=8, replace=False))
        Rc = Rf[cidx] + g.integers(30, 120, size=8)     # coarse pivots are fine pivots
        Gf = edge_set(grng.grng_edges(Kf, Rf))
        Gc = edge_set(grng.grng_edges(Kf[cidx], Rc))
        rel = grng.relative_membership(Kf[cidx], Rc, Kf, Rf)   # [mc, mf]
        for a in range(8):
            for b in range(8):
                if a == b or (min(a, b), max(a, b)) in Gc:
                    continue
                for i in np.nonzero(rel[a])[0]:
                    for j in np.nonzero(rel[b])[0]:
                        if i != j:
                            checks += 1
                            assert (min(i, j), max(i, j)) not in Gf
    assert checks > 0


def test_c_oracle_compact_and_upper_rows(oracle_native):
    """The bounded-memory row oracle equals the full-row one (rows longer than
    the first capacity are redone), and its upper rows are the full edge
    list's rows y > x."""
    W = synth.clustered(n=1500, d=8, clusters=4, m=0, q=19, sub=13)
    xs = np.arange(0, 1500, 11)
    full = oracle_native.rng_rows(W.X, W.q, xs)
    comp = oracle_native.rng_rows_compact(W.X, W.q, xs, cap=3)
    assert all(np.array_equal(a, b) for a, b in zip(full, comp))
    E = oracle_native.rng_edges(W.X, W.q)
    up = oracle_native.rng_rows_compact(W.X, W.q, xs, upper=True)
    for x, r in zip(xs, up):
        assert np.array_equal(r, np.sort(E[E[:, 0] == x, 1])), x
