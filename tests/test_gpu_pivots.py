"""Pivots added to built layers (dynamic pivot layers) on the GPU (needs an MI355X).

insert_pivots turns a layer's GRNG into GRNG(P u B): it must equal the
oracle's Definition 1 on the merged pivot set.  The exemplar RNG must stay the
oracle's, and insertions, queries and rebuilds after the change must stay
exact.  Orphan listing must equal the points outside every pivot domain
(exact squared distances on grid integers), and promoting orphans to pivots
must leave them parented.
"""
import numpy as np
import pytest

import synth
from oracle import native
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


def oracle_layer(X, q, ids, radii):
    return ids[native.grng_edges(X[ids], radii, q)]


def oracle_orphans(X, q, ids, radii):
    Xi = synth.grid_ints(X, q).astype(object)
    ri = [int(round(float(r) * 2.0 ** q)) for r in radii]
    P = Xi[ids]
    out = []
    for x in range(len(X)):
        d2 = ((P - Xi[x]) ** 2).sum(axis=1)
        if not any(d2[t] <= ri[t] * ri[t] for t in range(len(ids))):
            out.append(x)
    return np.array(out, dtype=np.int64)


def layer_edges(idx, layer):
    return idx.edges(layer).cpu().numpy().astype(np.int64)


@pytest.mark.parametrize("prec", [1, 2])
def test_inserted_pivots_give_the_merged_grng(G, prec):
    say("insert pivots into one layer, precision", prec)
    W = synth.clustered(n=4000, d=16, clusters=8, m=80, knn=40, sub=21)
    L = W.layers[0]
    g = np.random.default_rng(4)
    sel = g.permutation(len(L.pivot_ids))
    old, new = np.sort(sel[:60]), np.sort(sel[60:])
    idx = G.Index(to_dev(W.X), grid_exp=W.q, precision=prec)
    idx.build_grng_layer(0, to_dev(L.pivot_ids[old]), to_dev(L.radii[old]))
    idx.build_rng()
    E_rng = idx.edges().cpu().numpy().astype(np.int64)
    assert np.array_equal(layer_edges(idx, 0), oracle_layer(W.X, W.q, L.pivot_ids[old], L.radii[old]))
    idx.insert_pivots(0, to_dev(L.pivot_ids[new]), to_dev(L.radii[new]))
    assert np.array_equal(layer_edges(idx, 0), oracle_layer(W.X, W.q, L.pivot_ids, L.radii))
    assert np.array_equal(idx.edges().cpu().numpy().astype(np.int64), E_rng)
    assert np.array_equal(E_rng, native.rng_edges(W.X, W.q))
    # later work runs against the new pivots and stays exact
    B = synth.insert_batches(W, n_batches=1, lo=300, hi=301, sub=12)[0]
    idx.insert_batch(to_dev(B))
    U = np.vstack([W.X, B])
    assert np.array_equal(idx.edges().cpu().numpy().astype(np.int64), native.rng_edges(U, W.q))
    Q = synth.queries_like(W, 40, sub=5)
    off, nb = idx.query_neighbors(to_dev(Q))
    off, nb = off.cpu().numpy(), nb.cpu().numpy().astype(np.int64)
    for i, qp in enumerate(Q):
        assert np.array_equal(nb[off[i]:off[i + 1]], native.query_row(U, W.q, qp)), i
    idx.build_rng()
    assert np.array_equal(idx.edges().cpu().numpy().astype(np.int64), native.rng_edges(U, W.q))
    idx.close()


def test_promoted_orphans_are_parented(G):
    say("promote orphans to pivots")
    W = synth.clustered(n=3000, d=16, clusters=8, m=40, knn=12, sub=22)
    L = W.layers[0]
    idx = G.Index(to_dev(W.X), grid_exp=W.q, precision=1)
    idx.build_grng_layer(0, to_dev(L.pivot_ids), to_dev(L.radii))
    idx.build_rng()
    orph = idx.orphans().cpu().numpy().astype(np.int64)
    want = oracle_orphans(W.X, W.q, L.pivot_ids, L.radii)
    assert len(want) > 100
    assert np.array_equal(orph, want)
    assert idx.stats()["orphans"] == len(want)
    promote = np.sort(np.random.default_rng(2).choice(orph, 50, replace=False)).astype(np.int32)
    prad = synth.knn_radii(W.X, W.q, promote, 12)
    idx.insert_pivots(0, to_dev(promote), to_dev(prad))
    ids = np.concatenate([L.pivot_ids, promote])
    rad = np.concatenate([L.radii, prad])
    order = np.argsort(ids)
    ids, rad = ids[order].astype(np.int32), rad[order].astype(np.float32)
    assert np.array_equal(layer_edges(idx, 0), oracle_layer(W.X, W.q, ids, rad))
    after = idx.orphans().cpu().numpy().astype(np.int64)
    assert np.array_equal(after, oracle_orphans(W.X, W.q, ids, rad))
    assert not set(promote.tolist()) & set(after.tolist())
    B = synth.insert_batches(W, n_batches=1, lo=500, hi=501, sub=13)[0]
    idx.insert_batch(to_dev(B))
    assert np.array_equal(idx.edges().cpu().numpy().astype(np.int64), native.rng_edges(np.vstack([W.X, B]), W.q))
    idx.close()


def test_pivots_inserted_into_a_hierarchy(G):
    say("insert pivots into the coarse and the fine layer of a hierarchy")
    W = synth.subspace_layers(6000, ms=(30, 240))
    C, F = W.layers
    g = np.random.default_rng(6)
    keep = np.sort(g.choice(len(C.pivot_ids), 22, replace=False))
    add = np.setdiff1d(np.arange(len(C.pivot_ids)), keep)
    idx = G.Index(to_dev(W.X), grid_exp=W.q, precision=1)
    idx.build_grng_layer(0, to_dev(C.pivot_ids[keep]), to_dev(C.radii[keep]))
    # the fine layer without 30 of its non-coarse pivots
    fine_only = np.setdiff1d(np.arange(len(F.pivot_ids)), np.searchsorted(F.pivot_ids, C.pivot_ids))
    drop = np.sort(g.choice(fine_only, 30, replace=False))
    fk = np.setdiff1d(np.arange(len(F.pivot_ids)), drop)
    idx.build_grng_layer(1, to_dev(F.pivot_ids[fk]), to_dev(F.radii[fk]))
    idx.build_rng()
    E_rng = idx.edges().cpu().numpy().astype(np.int64)
    assert np.array_equal(E_rng, native.rng_edges(W.X, W.q))
    # a coarse pivot must already be a fine pivot
    with pytest.raises(G.GrngError) as e:
        idx.insert_pivots(0, to_dev(F.pivot_ids[drop[:1]]), to_dev(F.radii[drop[:1]]))
    assert e.value.status == -1
    # an existing pivot cannot be added again
    with pytest.raises(G.GrngError) as e:
        idx.insert_pivots(1, to_dev(F.pivot_ids[fk[:1]]), to_dev(F.radii[fk[:1]]))
    assert e.value.status == -1
    idx.insert_pivots(0, to_dev(C.pivot_ids[add]), to_dev(C.radii[add]))
    assert np.array_equal(layer_edges(idx, 0), oracle_layer(W.X, W.q, C.pivot_ids, C.radii))
    assert np.array_equal(layer_edges(idx, 1), oracle_layer(W.X, W.q, F.pivot_ids[fk], F.radii[fk]))
    idx.insert_pivots(1, to_dev(F.pivot_ids[drop]), to_dev(F.radii[drop]))
    assert np.array_equal(layer_edges(idx, 1), oracle_layer(W.X, W.q, F.pivot_ids, F.radii))
    assert np.array_equal(idx.edges().cpu().numpy().astype(np.int64), E_rng)
    idx.build_rng()
    assert np.array_equal(idx.edges().cpu().numpy().astype(np.int64), E_rng)
    idx.close()
