"""Pins of the RNG oracle against what the paper and the mathematics fix (CPU only).

Each pin is chosen so that a plausible mistake in the oracle (a "<=" for
"<", a dropped lune condition, a wrong index, a transposed operand) fails at
least one of them; ``test_pins_catch_planted_mistakes`` plants such mistakes in
copies of the oracle and checks that they are caught.
"""
import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components, minimum_spanning_tree

from oracle import exact, rng

ROOT_RNG = np.random.default_rng(20221012)


def edge_set(E):
    return {(int(u), int(v)) for u, v in np.asarray(E).reshape(-1, 2)}


def test_fp64_squared_distance_is_exact_on_the_grid():
    # The exactness premise: for grid integers below 2**24 in a dimension where
    # D * kmax^2 < 2**51, float64 evaluates d^2 exactly in any order and in
    # the ||a||^2 + ||b||^2 - 2 a.b form.  Checked against Python integers.
    g = np.random.default_rng(1)
    for d, kmax in [(2, 2 ** 24 - 1), (16, 6_300_000), (32, 2 ** 22), (96, 3_700_000)]:
        A = g.integers(-kmax, kmax + 1, size=(2000, d))
        B = g.integers(-kmax, kmax + 1, size=(2000, d))
        if d == 2:
            A = np.abs(A)
            B = np.abs(B)
        exact_vals = [exact.sqdist_py(a, b) for a, b in zip(A, B)]
        Af, Bf = A.astype(np.float64), B.astype(np.float64)
        seq = ((Af - Bf) ** 2).sum(axis=1)
        gemm = (Af * Af).sum(1) + (Bf * Bf).sum(1) - 2.0 * (Af * Bf).sum(1)
        assert [int(v) for v in seq] == exact_vals
        assert [int(v) for v in gemm] == exact_vals


def test_one_dimensional_points_give_the_sorted_path():
    # On a line, z strictly between u and v is always inside lune(u, v); the
    # RNG of distinct 1-D points is the path through them in sorted order.
    for n in (2, 3, 17, 64):
        k = ROOT_RNG.choice(10_000, size=n, replace=False).reshape(-1, 1).astype(np.int64)
        order = np.argsort(k[:, 0])
        want = {tuple(sorted((int(order[i]), int(order[i + 1])))) for i in range(n - 1)}
        assert edge_set(rng.rng_edges(k)) == want


def test_square_lattice_keeps_only_unit_edges():
    # Diagonals die (a corner is at distance 1 < sqrt 2 from both ends) and
    # longer axis pairs die (the midpoint); unit pairs have an empty lune.
    for side in (2, 3, 5):
        K = np.array([(i, j) for i in range(side) for j in range(side)], dtype=np.int64)
        E = edge_set(rng.rng_edges(K))
        want = {(a, b) for a in range(len(K)) for b in range(a + 1, len(K))
                if ((K[a] - K[b]) ** 2).sum() == 1}
        assert E == want
        assert len(E) == 2 * side * (side - 1)


def test_boundary_ties_keep_the_edge():
    # d((0,0),(3,4)) = 5 = d((0,0),(5,0)): the third point is on the lune's
    # boundary, not inside it (the definition uses ">="), so all three edges stay.
    K = np.array([[0, 0], [5, 0], [3, 4]], dtype=np.int64)
    assert edge_set(rng.rng_edges(K)) == {(0, 1), (0, 2), (1, 2)}
    # Strictly inside: (3,3) is at sqrt 18 and sqrt 13 from the ends of a length-5 pair.
    K = np.array([[0, 0], [5, 0], [3, 3]], dtype=np.int64)
    assert edge_set(rng.rng_edges(K)) == {(0, 2), (1, 2)}


def test_collinear_and_duplicates():
    K = np.array([[0, 0], [1, 0], [2, 0]], dtype=np.int64)
    assert edge_set(rng.rng_edges(K)) == {(0, 1), (1, 2)}
    # A duplicate pair has d = 0, so nothing is strictly closer: always linked;
    # and a duplicate never lies strictly inside its twin's lunes.
    K = np.array([[0], [0], [1]], dtype=np.int64)
    assert edge_set(rng.rng_edges(K)) == {(0, 1), (0, 2), (1, 2)}
    K = np.zeros((4, 3), dtype=np.int64)
    assert len(edge_set(rng.rng_edges(K))) == 6


def test_loops_implementation_agrees_on_tiny_inputs():
    g = np.random.default_rng(7)
    for trial in range(300):
        n = int(g.integers(1, 9))
        d = int(g.integers(1, 4))
        hi = 4 if trial % 2 else 1000      # small ranges create many exact ties
        K = g.integers(-hi, hi + 1, size=(n, d)).astype(np.int64)
        assert edge_set(rng.rng_edges(K)) == set(rng.rng_edges_loops(K))


def _mst_edges(K):
    D = exact.sqdist_rows(K, np.arange(len(K))).astype(np.float64)
    T = minimum_spanning_tree(csr_matrix(np.sqrt(D) + 1e-300 * (D == 0)))
    r, c = T.nonzero()
    return {tuple(sorted((int(a), int(b)))) for a, b in zip(r, c)}


@pytest.mark.parametrize("d", [2, 3, 5])
def test_containment_chain_mst_rng_gabriel(d):
    # 1NN subset MST subset RNG subset GG (Section 1); scipy's MST is an
    # independent textbook routine.  Continuous-valued inputs make the MST unique.
    g = np.random.default_rng(100 + d)
    K = g.integers(0, 2 ** 20, size=(150, d)).astype(np.int64)
    R = edge_set(rng.rng_edges(K))
    G = edge_set(rng.gabriel_edges(K))
    M = _mst_edges(K)
    assert M <= R <= G
    nn = rng.nearest_neighbour(K)
    assert {tuple(sorted((i, int(j)))) for i, j in enumerate(nn)} <= R
    A = np.zeros((len(K), len(K)))
    for u, v in R:
        A[u, v] = A[v, u] = 1
    assert connected_components(csr_matrix(A))[0] == 1


def test_invariances_permutation_translation_scaling():
    g = np.random.default_rng(11)
    K = g.integers(0, 300, size=(80, 3)).astype(np.int64)
    E = edge_set(rng.rng_edges(K))
    perm = g.permutation(len(K))
    Ep = edge_set(rng.rng_edges(K[perm]))
    assert {tuple(sorted((int(perm[u]), int(perm[v])))) for u, v in Ep} == E
    assert edge_set(rng.rng_edges(K + np.array([7, -3, 1000]))) == E
    assert edge_set(rng.rng_edges(K * 4)) == E


def test_query_row_matches_rng_of_the_union():
    g = np.random.default_rng(5)
    for _ in range(20):
        K = g.integers(0, 50, size=(40, 2)).astype(np.int64)
        Q = g.integers(0, 50, size=(1, 2)).astype(np.int64)
        U = np.vstack([K, Q])
        E = rng.rng_edges(U)
        want = sorted(int(u) for u, v in E if v == len(K)) + sorted(int(v) for u, v in E if u == len(K))
        assert sorted(rng.query_row(K, Q[0]).tolist()) == sorted(want)


def test_table4_average_degree_identity():
    rows = [ln.split() for ln in open(__file__.replace("test_oracle_rng.py", "golden/table4_real_data.txt"))
            if ln.strip() and not ln.startswith("#")]
    for name, n, links, deg in rows:
        assert round(rng.average_degree(int(links), int(n)), 4) == float(deg), name


# ---------------------------------------------------------------------------
# Planted mistakes: copies of the oracle with one plausible error each must
# fail at least one pin above.


def _mutant_le(K):          # "<=" instead of "<": boundary points would eliminate
    n = len(K)
    D = exact.sqdist_rows(K, np.arange(n))
    out = set()
    for u in range(n):
        for v in range(u + 1, n):
            w = (D[u] <= D[u, v]) & (D[v] <= D[u, v])
            w[[u, v]] = False
            if not w.any():
                out.add((u, v))
    return out


def _mutant_one_side(K):    # dropped second lune condition
    n = len(K)
    D = exact.sqdist_rows(K, np.arange(n))
    out = set()
    for u in range(n):
        for v in range(u + 1, n):
            w = D[u] < D[u, v]
            w[[u, v]] = False
            if not w.any():
                out.add((u, v))
    return out


def _mutant_transposed(K):  # wrong index: tests d(u,z) and d(u,v) against each other twice
    n = len(K)
    D = exact.sqdist_rows(K, np.arange(n))
    out = set()
    for u in range(n):
        for v in range(u + 1, n):
            w = (D[u] < D[u, v]) & (D[u] < D[v, u])
            w[[u, v]] = False
            if not w.any():
                out.add((u, v))
    return out


def test_pins_catch_planted_mistakes():
    tie = np.array([[0, 0], [5, 0], [3, 4]], dtype=np.int64)
    lattice = np.array([(i, j) for i in range(3) for j in range(3)], dtype=np.int64)
    good_tie = edge_set(rng.rng_edges(tie))
    good_lat = edge_set(rng.rng_edges(lattice))
    for mutant in (_mutant_le, _mutant_one_side, _mutant_transposed):
        caught = mutant(tie) != good_tie or mutant(lattice) != good_lat
        g = np.random.default_rng(3)
        K = g.integers(0, 2 ** 16, size=(60, 2)).astype(np.int64)
        caught = caught or not (_mst_edges(K) <= mutant(K))
        caught = caught or mutant(K) != edge_set(rng.rng_edges(K))
        assert caught, mutant.__name__
