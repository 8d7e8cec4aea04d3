"""GPU parity of query_neighbors and insert_batch against the oracle (needs an MI355X)."""
import numpy as np
import pytest

import synth
from oracle import exact, native, rng
from conftest import say

pytestmark = pytest.mark.gpu


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


def make_index(G, X, q, layer=None, precision=0):
    idx = G.Index(to_dev(X), grid_exp=q, precision=precision)
    if layer is not None:
        idx.build_grng_layer(0, to_dev(np.asarray(layer[0], np.int32)), to_dev(np.asarray(layer[1], np.float32)))
    idx.build_rng()
    return idx


def query_lists(idx, Q):
    off, nb = idx.query_neighbors(to_dev(Q))
    off = off.cpu().numpy()
    nb = nb.cpu().numpy().astype(np.int64)
    return [nb[off[i]:off[i + 1]] for i in range(len(Q))]


@pytest.mark.parametrize("layered,prec", [(True, 0), (True, 1), (True, 2), (False, 0)])
def test_query_neighbors_match_oracle(G, layered, prec):
    say("query", layered, "precision", prec)
    W = synth.clustered(n=2500, d=16, clusters=6, m=60, knn=40, sub=3)
    Q = synth.queries_like(W, 150)
    # plus: a duplicate of an indexed point and a far-away point
    Q = np.vstack([Q, W.X[17:18], np.full((1, 16), 20.0, np.float32)])
    idx = make_index(G, W.X, W.q, (W.layers[0].pivot_ids, W.layers[0].radii) if layered else None, prec)
    got = query_lists(idx, Q)
    idx.close()
    for i, qpt in enumerate(Q):
        want = native.query_row(W.X, W.q, qpt)
        assert np.array_equal(got[i], want), i


def test_query_capacity_protocol(G):
    say("query capacity")
    import ctypes as C
    W = synth.uniform2d(500)
    idx = make_index(G, W.X, W.q)
    Q = synth.uniform2d(40, sub=1).X
    import torch
    off = torch.empty(41, dtype=torch.int64, device="cuda")
    nb = torch.empty(1, dtype=torch.int32, device="cuda")
    needed = C.c_int64(0)
    st = G.lib().grng_query_neighbors(idx._h, C.c_void_p(to_dev(Q).data_ptr()), 40, C.c_void_p(off.data_ptr()),
                                      C.c_void_p(nb.data_ptr()), 1, C.byref(needed))
    assert st == -5 and needed.value > 1
    lists = query_lists(idx, Q)
    assert sum(len(l) for l in lists) == needed.value
    idx.close()


@pytest.mark.parametrize("layered,prec,lo,hi", [(True, 0, 100, 900), (True, 1, 100, 900), (False, 0, 100, 900),
                                               (True, 1, 10, 150), (True, 0, 10, 150), (True, 2, 100, 900),
                                               (True, 2, 10, 150)])
def test_insert_batches_match_rebuild_oracle(G, layered, prec, lo, hi):
    """Batches of 400 or more points into 50 pivot cells take the dense path
    (batch points in their cells' tiles); smaller ones the sparse path (the
    batch as the row side, tiles packed across cells)."""
    say("insert", layered, "precision", prec, "sizes", lo, hi)
    W = synth.clustered(n=2000, d=8, clusters=5, m=50, knn=30, sub=4)
    batches = synth.insert_batches(W, n_batches=3, lo=lo, hi=hi, sub=1)
    idx = make_index(G, W.X, W.q, (W.layers[0].pivot_ids, W.layers[0].radii) if layered else None, prec)
    allX = W.X
    for bi, B in enumerate(batches):
        idx.insert_batch(to_dev(B))
        allX = np.vstack([allX, B])
        got = idx.edges().cpu().numpy().astype(np.int64)
        want = native.rng_edges(allX, W.q)
        assert np.array_equal(got, want), bi
    st = idx.stats()
    assert st["n_points"] == len(allX)
    idx.close()


def test_insert_order_invariance_and_duplicates(G):
    say("insert order")
    W = synth.clustered(n=1500, d=4, clusters=4, m=40, knn=25, sub=5)
    b = synth.insert_batches(W, n_batches=2, lo=200, hi=400, sub=2)
    dup = W.X[:50].copy()            # exact duplicates of indexed points
    lay = (W.layers[0].pivot_ids, W.layers[0].radii)
    i1 = make_index(G, W.X, W.q, lay, precision=1)
    for B in (b[0], b[1], dup):
        i1.insert_batch(to_dev(B))
    e1 = i1.edges().cpu().numpy().astype(np.int64)
    i1.close()
    allX = np.vstack([W.X, b[0], b[1], dup])
    assert np.array_equal(e1, native.rng_edges(allX, W.q))
