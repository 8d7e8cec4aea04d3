"""Other metrics and empty-region graphs on the GPU (needs an MI355X).

The exhaustive path builds the RNG under the L1 and L-infinity distances, the
Euclidean Gabriel graph and lune-based beta-skeletons; edges, insertions and
query rows must equal the oracle's (rng_edges_metric, gabriel_edges,
beta_skeleton_edges, the graph of the union), including inputs on a coarse
integer grid full of exact ties and points on a lune's boundary at the largest
coordinates the grid contract allows.
"""
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import exact, rng
from conftest import say

pytestmark = pytest.mark.gpu

KINDS = [(1, 0, "l1"), (2, 0, "linf"), (0, 1, "gabriel"), (0, 2, "beta1.5"), (0, 2, "beta4")]


def beta_of(name):
    return float(name[4:]) if name.startswith("beta") else 0.0


@pytest.fixture(scope="module")
def G():
    import torch
    import paper_2208_10022_amd as P
    assert torch.cuda.is_available()
    P.lib()
    return P


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def oracle_edges(K, name):
    if name.startswith("beta"):
        return rng.beta_skeleton_edges(K, int(beta_of(name) * 4))
    return rng.gabriel_edges(K) if name == "gabriel" else rng.rng_edges_metric(K, name)


def inputs():
    g = np.random.default_rng(12)
    cases = [(synth.uniform2d(500, d=2, sub=1).X, 24), (synth.uniform2d(400, d=5, sub=2).X, 24),
             (synth.uniform2d(200, d=1, sub=3).X, 24),
             (g.integers(0, 10, size=(300, 2)).astype(np.float32), 0),      # exact ties everywhere
             (g.integers(0, 4, size=(120, 3)).astype(np.float32), 0)]
    return cases


@pytest.mark.parametrize("metric,graph,name", KINDS)
def test_exhaustive_graph_matches_oracle(G, metric, graph, name):
    for X, q in inputs():
        say(name, X.shape, "q", q)
        idx = G.Index(to_dev(X), grid_exp=q, metric=metric, graph=graph, beta=beta_of(name))
        idx.build_rng()
        got = idx.edges().cpu().numpy().astype(np.int64)
        idx.close()
        assert np.array_equal(got, oracle_edges(exact.to_grid(X, q), name)), (name, X.shape)


@pytest.mark.parametrize("metric,graph,name", KINDS)
def test_insert_and_query_match_oracle(G, metric, graph, name):
    say("insert/query", name)
    g = np.random.default_rng(5)
    X = g.integers(0, 200, size=(300, 3)).astype(np.float32)
    B = g.integers(0, 200, size=(80, 3)).astype(np.float32)
    Q = np.vstack([g.integers(0, 200, size=(20, 3)), X[:2]]).astype(np.float32)
    idx = G.Index(to_dev(X), grid_exp=0, metric=metric, graph=graph, beta=beta_of(name))
    idx.build_rng()
    idx.insert_batch(to_dev(B))
    U = np.vstack([X, B])
    assert np.array_equal(idx.edges().cpu().numpy().astype(np.int64), oracle_edges(exact.to_grid(U, 0), name))
    off, nb = idx.query_neighbors(to_dev(Q))
    off, nb = off.cpu().numpy(), nb.cpu().numpy().astype(np.int64)
    for i, qp in enumerate(Q):
        qi = len(U)
        if name.startswith("beta"):
            want = rng.beta_skeleton_row(exact.to_grid(np.vstack([U, qp[None]]), 0), qi, int(beta_of(name) * 4))
        else:
            E = oracle_edges(exact.to_grid(np.vstack([U, qp[None]]), 0), name)
            want = np.sort(np.concatenate([E[E[:, 1] == qi, 0], E[E[:, 0] == qi, 1]]))
        assert np.array_equal(np.sort(nb[off[i]:off[i + 1]]), want), (name, i)
    idx.close()


def test_pivot_layers_need_the_euclidean_rng(G):
    X = synth.uniform2d(100).X
    for metric, graph, name in KINDS:
        idx = G.Index(to_dev(X), grid_exp=24, metric=metric, graph=graph, beta=beta_of(name))
        with pytest.raises(G.GrngError) as e:
            idx.build_grng_layer(0, to_dev(np.arange(0, 100, 10, dtype=np.int32)),
                                 to_dev(np.zeros(10, np.float32)))
        assert e.value.status == -1, name
        idx.close()
    with pytest.raises(G.GrngError) as e:
        G.Index(to_dev(X), grid_exp=24, metric=1, graph=1)   # Gabriel is Euclidean only
    assert e.value.status == -1



def _boundary_cases():
    """(points, beta, pair kept?) at coordinates near 2^23: z on the boundary of
    one ball (kept: the balls are open) and one grid unit inside it (removed)."""
    u = 2 ** 20
    x, y = (-5 * u, 0), (5 * u, 0)
    # beta 2 (the RNG): |z - y| = |x - y| = 10u, a 6-8-10 triangle
    zr = (5 * u - 8 * u, 6 * u)
    # beta 3/2: ball around (2.5u, 0) of radius 7.5u; z = centre + (-4.5u, 6u)
    zb = (-2 * u, 6 * u)
    return [([x, y, zr], 2.0, True), ([x, y, (zr[0] + 1, zr[1])], 2.0, False),
            ([x, y, zb], 1.5, True), ([x, y, (zb[0] + 1, zb[1])], 1.5, False)]


def test_beta_skeleton_exact_at_large_coordinates(G):
    g = np.random.default_rng(9)
    for pts, beta, kept in _boundary_cases():
        say("beta boundary", beta, pts[2])
        # other points stay clear of the lune of (x, y) (|second coordinate| >= 9u)
        u = 2 ** 20
        extra = np.stack([g.integers(-15 * u, 15 * u, size=40),
                          g.integers(9 * u, 15 * u, size=40) * g.choice([-1, 1], size=40)], axis=1)
        K = np.vstack([np.array(pts, np.int64), extra]).astype(np.int64)
        idx = G.Index(to_dev(K.astype(np.float32)), grid_exp=0, graph=2, beta=beta)
        idx.build_rng()
        got = idx.edges().cpu().numpy().astype(np.int64)
        idx.close()
        want = rng.beta_skeleton_edges_loops(K, Fraction(beta))
        assert {tuple(e) for e in got.tolist()} == set(want)
        assert ((0, 1) in set(want)) == kept
