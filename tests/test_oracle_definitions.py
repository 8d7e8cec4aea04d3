"""Further pins of the oracle's definitions (CPU only).

* Definition 1 (Section 2) with unequal radii: the radius sums on the two
  sides of the generalized lune are (2 r_i + r_j) next to i and (r_i + 2 r_j)
  next to j.  A hand-computed layer fixes which side gets which sum.
* The Gabriel graph (Section 1, the proximity-graph chain): fixed cases with
  hand-computed edges, and the oracle against an independent formula of the
  same graph (the disk on the diameter uv is empty of points).
* The Stage VII bounds (Section 2, Proposition 5): mu_bar_max and mu_max on a
  hand-computed 1-D example, and the proposition itself as an implication
  between the oracle's insertion result and those bounds.
* The exactness contract of ``exact.to_grid``.
"""
import math

from fractions import Fraction

import numpy as np
import pytest

from oracle import exact, grng, rng


def edge_set(E):
    return {(int(u), int(v)) for u, v in np.asarray(E).reshape(-1, 2)}


# --- Definition 1 with unequal radii -----------------------------------------

F = 2 ** 20
# i = (0, 0) with r_i = 2F and j = (6F, 8F) with r_j = F, so d(i, j) = 10F.
# The G-lune of (i, j) holds k iff d(k, i) < 10F - (2 r_i + r_j) = 5F and
# d(k, j) < 10F - (r_i + 2 r_j) = 6F.  k = (3F, 4F - 1) has d(k, i)^2 =
# 25F^2 - 8F + 1 < (5F)^2 and d(k, j)^2 = 25F^2 + 8F + 1 < (6F)^2, so it blocks
# the link.  With the two sums exchanged (4F next to i, 5F next to j) it would
# not: d(k, j) > 5F.  The links (i, k) and (j, k) stay: their G-lunes are far
# too small to hold the third pivot (d(j, i) = 10F against thresholds of
# about F and 3F).
ASYM_P = np.array([[0, 0], [6 * F, 8 * F], [3 * F, 4 * F - 1]], np.int64)
ASYM_R = np.array([2 * F, F, 0], np.int64)


def test_asymmetric_radii_follow_definition1():
    assert edge_set(grng.grng_edges(ASYM_P, ASYM_R)) == {(0, 2), (1, 2)}
    # the same pivots listed in the other order: the link of the two radius
    # pivots is still blocked (Definition 1 is symmetric in i and j)
    perm = [1, 0, 2]
    assert edge_set(grng.grng_edges(ASYM_P[perm], ASYM_R[perm])) == {(0, 2), (1, 2)}
    # on the exact boundary d(k, i) = 5F the strict "<" keeps the link
    P = ASYM_P.copy()
    P[2] = (3 * F, 4 * F)
    assert edge_set(grng.grng_edges(P, ASYM_R)) == {(0, 1), (0, 2), (1, 2)}


def test_exchanged_radius_sums_fail_the_pin(monkeypatch):
    """A plausible slip, the two radius sums exchanged, is caught by the pin."""
    def swapped(d2_ki, d2_kj, d2_ij, ri, rj):
        return exact.sqrt_plus_lt(d2_ki, ri + 2 * rj, d2_ij) and exact.sqrt_plus_lt(d2_kj, 2 * ri + rj, d2_ij)
    monkeypatch.setattr(grng, "in_glune", swapped)
    assert edge_set(grng.grng_edges(ASYM_P, ASYM_R)) != {(0, 2), (1, 2)}


def test_c_oracle_agrees_on_asymmetric_radii(oracle_native):
    X = ASYM_P.astype(np.float32)
    got = oracle_native.grng_edges(X, ASYM_R.astype(np.float32), 0)
    assert edge_set(got) == {(0, 2), (1, 2)}


# --- Gabriel graph -----------------------------------------------------------

@pytest.mark.parametrize("pts,want", [
    # (2,1) sees u=(0,0), v=(4,0) at an obtuse angle: inside the diameter disk
    ([[0, 0], [4, 0], [2, 1]], {(0, 2), (1, 2)}),
    # (2,3): acute angle, outside the disk, so all three are Gabriel edges
    ([[0, 0], [4, 0], [2, 3]], {(0, 1), (0, 2), (1, 2)}),
    # (1,1) on the circle with diameter (0,0)-(2,0): boundary keeps the edge
    ([[0, 0], [2, 0], [1, 1]], {(0, 1), (0, 2), (1, 2)}),
    # a square: each diagonal has the other two corners on its circle
    ([[0, 0], [1, 0], [1, 1], [0, 1]], {(0, 1), (1, 2), (2, 3), (0, 3), (0, 2), (1, 3)}),
    # collinear: the middle point blocks the long pair
    ([[0, 0], [1, 0], [2, 0]], {(0, 1), (1, 2)}),
])
def test_gabriel_fixed_cases(pts, want):
    assert edge_set(rng.gabriel_edges(np.array(pts, np.int64))) == want


def _gabriel_by_midpoint_disk(K):
    """Independent formula: z blocks (u, v) iff |2z - u - v| < |u - v| (open disk
    centred at the midpoint with radius d(u,v)/2), in Python integers."""
    pts = [tuple(int(c) for c in row) for row in K]
    n = len(pts)
    out = set()
    for u in range(n):
        for v in range(u + 1, n):
            duv = sum((a - b) ** 2 for a, b in zip(pts[u], pts[v]))
            ok = True
            for z in range(n):
                if z in (u, v):
                    continue
                m = sum((2 * c - a - b) ** 2 for c, a, b in zip(pts[z], pts[u], pts[v]))
                if m < duv:
                    ok = False
                    break
            if ok:
                out.add((u, v))
    return out


def test_gabriel_matches_the_midpoint_disk_formula():
    g = np.random.default_rng(31)
    for t in range(40):
        n = int(g.integers(3, 25))
        d = int(g.integers(1, 4))
        K = g.integers(0, 6 if t % 2 else 1000, size=(n, d)).astype(np.int64)   # small grids force ties
        assert edge_set(rng.gabriel_edges(K)) == _gabriel_by_midpoint_disk(K)


def test_rng_is_strictly_inside_gabriel_on_a_fixed_case():
    K = np.array([[0, 0], [4, 0], [2, 3]], np.int64)
    assert edge_set(rng.rng_edges(K)) == {(0, 2), (1, 2)}
    assert edge_set(rng.gabriel_edges(K)) == {(0, 1), (0, 2), (1, 2)}


# --- lune-based beta-skeleton ---------------------------------------------------

# u = (0,0), v = (40,0), beta = 3/2: the balls have radius 30 around (30,0) and
# (10,0), so z = (20,28) (10^2 + 28^2 = 884 < 900) blocks (u, v) and z = (20,29)
# (941 > 900) does not; the RNG lune (radius 40 around u and v) holds both.
@pytest.mark.parametrize("z,beta,want", [
    ((20, 28), Fraction(3, 2), {(0, 2), (1, 2)}),
    ((20, 29), Fraction(3, 2), {(0, 1), (0, 2), (1, 2)}),
    ((20, 29), Fraction(2), {(0, 2), (1, 2)}),
    ((20, 29), Fraction(1), {(0, 1), (0, 2), (1, 2)}),
    # (20, 20) lies on the Gabriel circle of (u, v): the open disk keeps the edge
    ((20, 20), Fraction(1), {(0, 1), (0, 2), (1, 2)}),
    ((20, 20), Fraction(5, 4), {(0, 2), (1, 2)}),
])
def test_beta_skeleton_fixed_cases(z, beta, want):
    K = np.array([[0, 0], [40, 0], list(z)], np.int64)
    assert edge_set(rng.beta_skeleton_edges(K, int(beta * 4))) == want
    assert set(rng.beta_skeleton_edges_loops(K, beta)) == want


def test_beta_skeleton_special_cases_and_nesting():
    # beta 1 is the Gabriel graph and beta 2 the RNG (both pinned above by
    # their own fixed cases); a larger beta widens the region, so the graphs
    # nest; on a line every beta >= 1 leaves the sorted path.
    g = np.random.default_rng(41)
    for t in range(12):
        n, d = int(g.integers(5, 40)), int(g.integers(1, 4))
        K = g.integers(0, 5 if t % 3 == 0 else 10 ** 5, size=(n, d)).astype(np.int64)
        assert edge_set(rng.beta_skeleton_edges(K, 4)) == edge_set(rng.gabriel_edges(K))
        assert edge_set(rng.beta_skeleton_edges(K, 8)) == edge_set(rng.rng_edges(K))
        prev = None
        for a in (4, 5, 6, 8, 11, 16, 64):
            E = edge_set(rng.beta_skeleton_edges(K, a))
            if prev is not None:
                assert E <= prev, (t, a)
            prev = E
    x = np.unique(g.integers(0, 1000, size=30))
    K = x[g.permutation(len(x))][:, None].astype(np.int64)
    order = np.argsort(K[:, 0])
    path = {tuple(sorted((int(order[i]), int(order[i + 1])))) for i in range(len(order) - 1)}
    for a in (4, 6, 8, 13, 64):
        assert edge_set(rng.beta_skeleton_edges(K, a)) == path


def test_beta_skeleton_on_a_ball_boundary_at_large_coordinates():
    # x = (-5u, 0), y = (5u, 0), u = 2^20.  beta 2: z = (-3u, 6u) has |z - y| =
    # 10u = |x - y| (a 6-8-10 triangle), on the boundary; one unit toward y it
    # is inside.  beta 3/2: the ball around (2.5u, 0) has radius 7.5u and
    # z = (-2u, 6u) lies on it (4.5^2 + 6^2 = 7.5^2), while |z - (-2.5u, 0)|^2 =
    # 36.25 u^2 < 56.25 u^2 puts it inside the other ball.
    u = 2 ** 20
    for z, beta in (((-3 * u, 6 * u), Fraction(2)), ((-2 * u, 6 * u), Fraction(3, 2))):
        on = np.array([[-5 * u, 0], [5 * u, 0], list(z)], np.int64)
        inside = on.copy()
        inside[2, 0] += 1
        assert set(rng.beta_skeleton_edges_loops(on, beta)) == {(0, 1), (0, 2), (1, 2)}
        assert set(rng.beta_skeleton_edges_loops(inside, beta)) == {(0, 2), (1, 2)}


def test_beta_skeleton_rows_match_the_edge_set():
    g = np.random.default_rng(47)
    for t in range(6):
        K = g.integers(0, 8 if t % 2 else 500, size=(30, 2)).astype(np.int64)
        a = int(g.integers(4, 20))
        E = rng.beta_skeleton_edges(K, a)
        for i in range(len(K)):
            want = np.sort(np.concatenate([E[E[:, 1] == i, 0], E[E[:, 0] == i, 1]]))
            assert np.array_equal(rng.beta_skeleton_row(K, i, a), want), (t, i)


def test_beta_skeleton_integer_form_matches_the_rational_centres():
    g = np.random.default_rng(43)
    for t in range(25):
        n, d = int(g.integers(3, 12)), int(g.integers(1, 4))
        K = g.integers(0, 4 if t % 2 else 50, size=(n, d)).astype(np.int64)
        a = int(g.integers(4, 30))
        assert edge_set(rng.beta_skeleton_edges(K, a)) == set(rng.beta_skeleton_edges_loops(K, Fraction(a, 4))), t


# --- Stage VII bounds (Proposition 5) -----------------------------------------

def test_mu_bounds_on_a_hand_computed_line():
    # points 0, 1, 3, 7 on a line: the RNG is the path 0-1-3-7 with lengths 1, 2, 4
    K = np.array([[0], [1], [3], [7]], np.int64)
    E = rng.rng_edges(K)
    assert edge_set(E) == {(0, 1), (1, 2), (2, 3)}
    mb = grng.mu_bar_max_sq(4, K, E)
    assert mb.tolist() == [1, 4, 16, 16]
    # pivot at point 1 (coordinate 1) with radius 2 holds coordinates 0, 1, 3:
    #   mu_max = max(1 + 1, 2 + 0, 4 + 2) = 6
    # pivot at point 3 (coordinate 7) with radius 0 holds only itself: 4 + 0
    # pivot at point 0 (coordinate 0) with radius 3 holds 0, 1, 3: max(1, 2+1, 4+3) = 7
    mu = grng.mu_max(K, [1, 3, 0], [2, 0, 3], mb)
    assert mu.tolist() == [6.0, 4.0, 7.0]


def test_mu_bar_of_an_isolated_point_is_zero():
    K = np.array([[0, 0]], np.int64)
    assert grng.mu_bar_max_sq(1, K, np.zeros((0, 2), np.int64)).tolist() == [0]


@pytest.mark.parametrize("seed", range(6))
def test_proposition5_bounds_never_skip_an_invalidated_edge(seed):
    """Adding Q to S removes exactly the edges of RNG(S) whose lune holds Q.
    Proposition 5: no edge at x is removed when d(Q, x) >= mu_bar_max(x), and
    none at any member of pivot p when d(Q, p) >= mu_max(p).  Both skips are
    checked against the oracle's rebuild, and must fire for some (Q, x)."""
    g = np.random.default_rng(100 + seed)
    n, d = 60, 2
    K = g.integers(0, 400, size=(n, d)).astype(np.int64)
    E = rng.rng_edges(K)
    es = edge_set(E)
    mb = grng.mu_bar_max_sq(n, K, E)
    pid = g.choice(n, 8, replace=False)
    R = g.integers(20, 120, size=8)
    mu = grng.mu_max(K, pid, R, mb)
    member = grng.membership(K, pid, R)
    fired_x = fired_p = removed = 0
    for _ in range(40):
        q = g.integers(-50, 450, size=(1, d)).astype(np.int64)
        after = edge_set(rng.rng_edges(np.vstack([K, q])))
        gone = {e for e in es if e not in after}
        removed += len(gone)
        dq2 = ((K - q) ** 2).sum(axis=1)
        touched = {u for e in gone for u in e}
        for x in range(n):
            if dq2[x] >= mb[x]:          # d(Q,x) >= mu_bar_max(x), on squares
                fired_x += 1
                assert x not in touched
        dqp = np.sqrt(((K[pid] - q) ** 2).sum(axis=1).astype(np.float64))
        for t in range(len(pid)):
            if np.isfinite(mu[t]) and dqp[t] >= mu[t] * (1 + 1e-12):
                fired_p += 1
                assert not (set(np.nonzero(member[:, t])[0].tolist()) & touched)
    assert removed > 0 and fired_x > 0 and fired_p > 0


def test_mu_pins_catch_planted_mistakes(monkeypatch):
    K = np.array([[0], [1], [3], [7]], np.int64)
    E = rng.rng_edges(K)
    mb = grng.mu_bar_max_sq(4, K, E)
    good = grng.mu_max(K, [1, 3, 0], [2, 0, 3], mb).tolist()

    def mu_no_offset(K_, pivot_ids, R, mu_bar_sq):   # the d(x, p) term dropped
        M = grng.membership(K_, pivot_ids, R)
        val = np.sqrt(mu_bar_sq.astype(np.float64))[:, None] + 0.0 * M
        return np.where(M, val, -math.inf).max(axis=0)
    assert mu_no_offset(K, [1, 3, 0], [2, 0, 3], mb).tolist() != good


# --- exactness contract --------------------------------------------------------

def test_to_grid_enforces_the_contract():
    assert exact.to_grid(np.array([[2.0 ** 24 - 1]]), 0).tolist() == [[2 ** 24 - 1]]
    with pytest.raises(ValueError):
        exact.to_grid(np.array([[2.0 ** 24]]), 0)
    with pytest.raises(ValueError):
        exact.to_grid(np.array([[0.5]]), 0)          # off the grid
    # d * kmax^2 < 2^51: 2^23 in 32 dimensions is 2^51, one too many
    ok = np.full((1, 31), 2.0 ** 23)
    assert exact.to_grid(ok, 0).shape == (1, 31)
    with pytest.raises(ValueError):
        exact.to_grid(np.full((1, 32), 2.0 ** 23), 0)


# --- other metrics (RNG under L1 and L-infinity) -------------------------------

def test_metric_rng_hand_computed_case():
    # u=(0,0), v=(4,0), z=(2,2): d_1(u,z) = 4 is not below d_1(u,v) = 4, so
    # under L1 all three pairs are linked; under L-infinity d(u,z) = 2 < 4 and
    # z removes (u,v); Euclidean: sqrt(8) < 4, the same as L-infinity.
    K = np.array([[0, 0], [4, 0], [2, 2]], np.int64)
    assert edge_set(rng.rng_edges_metric(K, "l1")) == {(0, 1), (0, 2), (1, 2)}
    assert edge_set(rng.rng_edges_metric(K, "linf")) == {(0, 2), (1, 2)}
    assert edge_set(rng.rng_edges_metric(K, "l2sq")) == edge_set(rng.rng_edges(K))


@pytest.mark.parametrize("metric", ["l1", "linf"])
def test_metric_rng_pins(metric):
    g = np.random.default_rng(41)
    # 1-D: every metric is |a - b|, so the RNG is the sorted path
    x = g.permutation(40)[:25].astype(np.int64).reshape(-1, 1)
    order = np.argsort(x[:, 0])
    path = {tuple(sorted((int(order[i]), int(order[i + 1])))) for i in range(len(order) - 1)}
    assert edge_set(rng.rng_edges_metric(x, metric)) == path
    # loop-only implementation agrees on tiny inputs with many ties
    for t in range(120):
        n = int(g.integers(1, 8))
        K = g.integers(0, 4 if t % 2 else 500, size=(n, int(g.integers(1, 4)))).astype(np.int64)
        assert edge_set(rng.rng_edges_metric(K, metric)) == set(rng.rng_edges_metric_loops(K, metric))
    # the metric's minimum spanning tree (scipy, an independent routine) lies in the RNG
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import minimum_spanning_tree
    K = g.integers(0, 2 ** 20, size=(120, 3)).astype(np.int64)
    D = rng.metric_dists(K, metric).astype(np.float64)
    T = minimum_spanning_tree(csr_matrix(D + 1e-300 * (D == 0)))
    r, c = T.nonzero()
    assert {tuple(sorted((int(a), int(b)))) for a, b in zip(r, c)} <= edge_set(rng.rng_edges_metric(K, metric))
