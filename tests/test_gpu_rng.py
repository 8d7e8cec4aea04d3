"""GPU parity of the exact RNG / GRNG build against the oracle (needs an MI355X).

Edge sets must be identical (integer output: bit-exact).  Every case runs
through the C ABI via the Python binding.
"""
import os

import numpy as np
import pytest

import synth
from oracle import exact, native, rng
from conftest import say

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def G():
    import torch
    import paper_2208_10022_amd as P
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    P.lib()
    return P


# Every arithmetic form must give identical edges: float64 everywhere (0),
# float32 screens with exact float64 re-decision (1), and bf16 MFMA distance
# tiles with a per-tile error bound in the pair kernel (2).
PRECISIONS = [0, 1, 2]


def golden_edges(name):
    rows = [ln.split() for ln in open(os.path.join(HERE, "golden", name)) if ln.strip() and not ln.startswith("#")]
    return np.array(rows, dtype=np.int64).reshape(-1, 2)


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def gpu_edges(G, X, q, layers=(), **kw):
    idx = G.Index(to_dev(X), grid_exp=q, **kw)
    for l, (pid, rad) in enumerate(layers):
        idx.build_grng_layer(l, to_dev(np.asarray(pid, np.int32)), to_dev(np.asarray(rad, np.float32)))
    idx.build_rng()
    E = idx.edges().cpu().numpy().astype(np.int64)
    lay = [idx.edges(l).cpu().numpy().astype(np.int64) for l in range(len(layers))]
    st = idx.stats()
    idx.close()
    return E, lay, st


def test_uniform2d_1000_bruteforce_matches_golden(G):
    say("uniform2d n=1000 brute force")
    W = synth.uniform2d(1000)
    E, _, st = gpu_edges(G, W.X, W.q)
    want = golden_edges("uniform2d_n1000_rng_edges.txt")
    assert np.array_equal(E, want)
    assert st["n_edges"] == len(want)


def test_uniform2d_1000_guided_matches_golden(G):
    say("uniform2d n=1000 with a 40-pivot layer")
    W = synth.uniform2d(1000)
    g = np.random.default_rng(3)
    pid = np.sort(g.choice(1000, 40, replace=False)).astype(np.int32)
    rad = synth.knn_radii(W.X, W.q, pid, 25)
    E, lay, _ = gpu_edges(G, W.X, W.q, [(pid, rad)])
    assert np.array_equal(E, golden_edges("uniform2d_n1000_rng_edges.txt"))
    assert np.array_equal(lay[0], pid[native.grng_edges(W.X[pid], rad, W.q)])


@pytest.mark.parametrize("prec", PRECISIONS)
def test_clustered_3000_d16_matches_golden(G, prec):
    say("clustered n=3000 d=16 m=60 precision", prec)
    W = synth.clustered(n=3000, d=16, clusters=8, m=60, knn=40)
    L = W.layers[0]
    E, lay, st = gpu_edges(G, W.X, W.q, [(L.pivot_ids, L.radii)], precision=prec)
    assert np.array_equal(E, golden_edges("clustered_n3000_d16_rng_edges.txt"))
    assert np.array_equal(lay[0], L.pivot_ids[golden_edges("clustered_n3000_d16_m60_grng_edges.txt")])
    assert st["candidate_pairs"] > 0


@pytest.mark.parametrize("prec", PRECISIONS)
def test_lune_visit_order_keeps_edges(G, prec):
    """Visiting a pair's witness cells by max(d(x,p), d(y,p)) instead of
    d(x,p) changes only the number of witness tests."""
    say("lune visit order, precision", prec)
    W = synth.clustered(n=3000, d=16, clusters=8, m=60, knn=40)
    L = W.layers[0]
    E0, _, s0 = gpu_edges(G, W.X, W.q, [(L.pivot_ids, L.radii)], precision=prec)
    E, _, st = gpu_edges(G, W.X, W.q, [(L.pivot_ids, L.radii)], precision=prec, witness_order=G.ORDER_LUNE)
    assert np.array_equal(E, golden_edges("clustered_n3000_d16_rng_edges.txt"))
    assert np.array_equal(E, E0)
    assert st["exhaustive_pairs"] == s0["exhaustive_pairs"] and st["lune_tests"] > 0
    W = synth.clustered(n=900, d=96, clusters=3, m=24, knn=30, q=18, sub=8)
    L = W.layers[0]
    E, _, _ = gpu_edges(G, W.X, W.q, [(L.pivot_ids, L.radii)], precision=prec, witness_order=G.ORDER_LUNE)
    assert np.array_equal(E, native.rng_edges(W.X, W.q))


@pytest.mark.parametrize("n,d,m,clusters,seed", [
    (1037, 2, 30, 4, 0), (2111, 3, 70, 6, 1), (1500, 5, 16, 3, 2), (777, 16, 100, 5, 3),
    (2049, 7, 64, 9, 4), (300, 1, 10, 2, 5), (1900, 12, 1, 4, 6), (650, 33, 20, 3, 7),
    (900, 96, 24, 3, 8), (500, 100, 10, 2, 9),
    # largest dimension of the tiled path (its LDS rows); two pivots leave
    # about half of all pairs to Stage V
    (600, 104, 2, 1, 10)])
@pytest.mark.parametrize("prec", PRECISIONS)
def test_guided_and_bruteforce_match_oracle_ragged(G, n, d, m, clusters, seed, prec):
    say("ragged", n, d, m, clusters, seed, "precision", prec)
    # 2^-18 grid above 64 dimensions keeps d * kmax^2 below 2^51
    W = synth.clustered(n=n, d=d, clusters=clusters, m=m, knn=min(30, n - 1), q=18 if d > 64 else 19, sub=seed)
    L = W.layers[0]
    want = native.rng_edges(W.X, W.q)
    E, lay, _ = gpu_edges(G, W.X, W.q, [(L.pivot_ids, L.radii)], precision=prec)
    assert np.array_equal(E, want)
    assert np.array_equal(lay[0], L.pivot_ids[native.grng_edges(W.X[L.pivot_ids], L.radii, W.q)])
    Eb, _, _ = gpu_edges(G, W.X, W.q, precision=prec)
    assert np.array_equal(Eb, want)


def test_witness_pivot_counts_do_not_change_edges(G):
    """Stage IV pivot witnesses (1..16) and Proposition 1 witness pivots per
    block (1 .. all) only change how much is pruned, never the edges."""
    say("witness pivot count sweep")
    W = synth.clustered(n=2500, d=8, clusters=6, m=80, knn=30, sub=11)
    L = W.layers[0]
    want = native.rng_edges(W.X, W.q)
    for k in (1, 4, 9, 16):
        E, _, _ = gpu_edges(G, W.X, W.q, [(L.pivot_ids, L.radii)], stage4_pivots=k)
        assert np.array_equal(E, want), k
    cands = []
    for kw in (1, 5, 33, 80, 500):
        E, _, st = gpu_edges(G, W.X, W.q, [(L.pivot_ids, L.radii)], vgrng_pivots=kw)
        assert np.array_equal(E, want), kw
        cands.append(st["candidate_pairs"])
    # more witnesses prune at least as much (all pivots at 80 and beyond)
    assert cands[0] >= cands[2] >= cands[3] == cands[4]


def test_autotune_keeps_edges_and_tunes_once(G):
    say("autotune, clustered n=3000 m=60")
    W = synth.clustered(n=3000, d=16, clusters=8, m=60, knn=40)
    L = W.layers[0]
    idx = G.Index(to_dev(W.X), grid_exp=W.q, autotune=1)
    idx.build_grng_layer(0, to_dev(L.pivot_ids), to_dev(L.radii))
    idx.build_rng()
    st = idx.stats()
    assert np.array_equal(idx.edges().cpu().numpy().astype(np.int64), golden_edges("clustered_n3000_d16_rng_edges.txt"))
    assert st["ms_autotune"] > 0 and st["vgrng_pivots"] in (60,) and st["stage4_pivots"] in (8, 12, 16)
    idx.build_rng()   # tuned once per index
    st2 = idx.stats()
    assert st2["ms_autotune"] == st["ms_autotune"] and st2["vgrng_pivots"] == st["vgrng_pivots"]
    idx.close()


@pytest.mark.parametrize("prec", PRECISIONS)
def test_partner_pass_only_removes_non_edges(G, prec):
    """Stage V with the row's other candidates: every pair it removes is a
    non-edge (the edge set stays the oracle's), and it removes most of them."""
    say("partner pass, clustered n=3000, precision", prec)
    W = synth.clustered(n=3000, d=16, clusters=8, m=60, knn=40)
    L = W.layers[0]
    idx = G.Index(to_dev(W.X), grid_exp=W.q, precision=prec)
    idx.build_grng_layer(0, to_dev(L.pivot_ids), to_dev(L.radii))
    idx.build_rng()
    st = idx.stats()
    assert np.array_equal(idx.edges().cpu().numpy().astype(np.int64), golden_edges("clustered_n3000_d16_rng_edges.txt"))
    left = st["exhaustive_pairs"] - st["partner_kills"]
    assert st["n_edges"] <= left   # the edges are among the pairs the scan decides
    assert st["partner_kills"] > 0.5 * (st["exhaustive_pairs"] - st["n_edges"])
    assert st["partner_tests"] > 0 and st["ms_partner"] > 0
    idx.close()


def test_autotune_chooses_the_tile_shape(G):
    """GRNG_PREC_AUTO: the autotuner times the float64-tile and the bf16-tile
    forms and keeps one; without the autotuner the padded dimension decides."""
    say("automatic tile shape, subspace n=6000 d=32")
    W = synth.subspace_layers(6000, ms=(30, 240))
    want = native.rng_edges(W.X, W.q)
    idx = G.Index(to_dev(W.X), grid_exp=W.q, precision=G.PREC_AUTO, autotune=1)
    for l, L in enumerate(W.layers):
        idx.build_grng_layer(l, to_dev(L.pivot_ids), to_dev(L.radii))
    idx.build_rng()
    st = idx.stats()
    assert st["precision_used"] in (G.PREC_FP32, G.PREC_BF16) and st["ms_autotune"] > 0
    assert np.array_equal(idx.edges().cpu().numpy().astype(np.int64), want)
    idx.build_rng()   # the choice is kept
    assert idx.stats()["precision_used"] == st["precision_used"]
    assert np.array_equal(idx.edges().cpu().numpy().astype(np.int64), want)
    idx.close()
    W16 = synth.clustered(n=2000, d=16, clusters=8, m=40, knn=40)
    for X, q, d_used in ((W.X, W.q, G.PREC_BF16), (W16.X, W16.q, G.PREC_FP32)):
        idx = G.Index(to_dev(X), grid_exp=q, precision=G.PREC_AUTO)
        idx.build_rng()   # no layer: the exhaustive path, form from the padded dimension
        assert idx.stats()["precision_used"] == d_used
        idx.close()


@pytest.mark.parametrize("prec", PRECISIONS)
def test_degenerate_inputs(G, prec):
    say("degenerate inputs precision", prec)
    # one point, two points, all identical, 1-D path, boundary tie, collinear.
    cases = [np.zeros((1, 3), np.float32), np.array([[0, 0], [1, 2]], np.float32),
             np.zeros((7, 4), np.float32),
             np.array([[5], [1], [9], [3], [7]], np.float32),
             np.array([[0, 0], [5, 0], [3, 4]], np.float32),
             np.array([[0, 0], [1, 0], [2, 0]], np.float32),
             np.array([[0], [0], [1]], np.float32)]
    for X in cases:
        want = rng.rng_edges(exact.to_grid(X, 0))
        E, _, _ = gpu_edges(G, X, 0, precision=prec)
        assert np.array_equal(E, want), X
        if len(X) >= 3:   # same with every point a zero-radius pivot (GRNG = RNG, Section 2)
            pid = np.arange(len(X), dtype=np.int32)
            E2, lay, _ = gpu_edges(G, X, 0, [(pid, np.zeros(len(X), np.float32))], precision=prec)
            assert np.array_equal(E2, want)
            assert np.array_equal(lay[0], want)


@pytest.mark.parametrize("prec", PRECISIONS)
def test_grid_lattice_with_pivots(G, prec):
    say("lattice 20x20 with pivots precision", prec)
    K = np.array([(i, j) for i in range(20) for j in range(20)], np.float32)
    pid = np.arange(0, 400, 7, dtype=np.int32)
    E, lay, _ = gpu_edges(G, K, 0, [(pid, np.full(len(pid), 2.0, np.float32))], precision=prec)
    assert len(E) == 2 * 20 * 19
    assert np.array_equal(E, rng.rng_edges(exact.to_grid(K, 0)))


def test_error_statuses(G):
    say("error statuses")
    import torch
    X = to_dev(np.array([[0.5, 0.25], [0.1, 0.3]], np.float32))
    with pytest.raises(G.GrngError) as e:
        G.Index(X, grid_exp=1)           # 0.1 is not a multiple of 2^-1
    assert e.value.status == -4
    Xn = to_dev(np.array([[0.0, np.nan]], np.float32))
    with pytest.raises(G.GrngError) as e:
        G.Index(Xn, grid_exp=4)
    assert e.value.status == -4
    W = synth.uniform2d(200)
    idx = G.Index(to_dev(W.X), grid_exp=W.q)
    with pytest.raises(G.GrngError) as e:
        idx.build_grng_layer(1, to_dev(np.array([1, 2], np.int32)), to_dev(np.array([0.1, 0.1], np.float32)))
    assert e.value.status == -6
    with pytest.raises(G.GrngError) as e:
        idx.build_grng_layer(0, to_dev(np.array([2, 1], np.int32)), to_dev(np.array([0.0, 0.0], np.float32)))
    assert e.value.status == -1
    with pytest.raises(G.GrngError) as e:
        idx.edges()
    assert e.value.status == -6
    idx.build_rng()
    assert idx.num_edges() == len(rng.rng_edges(exact.to_grid(W.X, W.q)))
    idx.close()
    del torch


def test_witness_cells_beyond_the_sort_capacity(G):
    """4,500 pivots and one far outlier: the outlier's pairs are long, so every
    cell may hold a witness for them and its cell list (more than the 4,096
    entries sorted in LDS) is scanned in pivot order.  Sampled rows, the
    outlier's among them, equal the oracle's."""
    say("4500 pivots with a far outlier n=12001 d=3")
    W = synth.clustered(n=12000, d=3, clusters=6, m=4500, knn=8, sub=21)
    X = np.vstack([W.X, np.full((1, 3), 25.0, np.float32)])   # 25 * 2^19 < 2^24: on the grid
    pid = W.layers[0].pivot_ids
    rad = synth.knn_radii(X, W.q, pid, 8)
    E, _, st = gpu_edges(G, X, W.q, [(pid, rad)])
    say("stats", st)
    assert st["unsorted_cell_rows"] > 0   # the pivot-order path ran
    g = np.random.default_rng(5)
    xs = np.concatenate([[X.shape[0] - 1], g.choice(W.n, 12, replace=False)])
    rows = native.rng_rows(X, W.q, xs)
    assert len(rows[0]) > 0
    for x, row in zip(xs, rows):
        got = np.sort(np.concatenate([E[E[:, 0] == x, 1], E[E[:, 1] == x, 0]]))
        assert np.array_equal(got, row), x


def test_float32_screen_redecides_exact_ties(G):
    """3-4-5 triangles A=(0,0), B=(5,0), C=(3,4) far apart: for the pair
    (A, B) the point C sits exactly on the lune boundary (d(A,C) = d(A,B) = 5),
    so the edge is kept (strict lune) and the float32 screen cannot decide C:
    those comparisons must be re-decided in float64."""
    say("float32 screen on exact ties")
    g = np.random.default_rng(5)
    offs = np.unique(g.integers(0, 60, size=(80, 2)), axis=0)[:50] * 100
    tri = np.array([[0, 0], [5, 0], [3, 4]])
    P = (offs[:, None, :] + tri[None, :, :]).reshape(-1, 2).astype(np.float32)
    pid = np.arange(2, len(P), 3, dtype=np.int32)      # each C is a pivot of radius 5
    rad = np.full(len(pid), 5.0, np.float32)
    want = rng.rng_edges(exact.to_grid(P, 0))
    for prec in PRECISIONS:
        E, _, st = gpu_edges(G, P, 0, [(pid, rad)], precision=prec)
        assert np.array_equal(E, want), prec
        if prec >= 1:
            assert st["rechecks"] > 0
        else:
            assert st["rechecks"] == 0


def test_grng_layer_exact_ties_use_the_integer_predicate(G):
    """G-lune ties at large coordinates (Definition 1 uses a strict "<"):
    k = (3F, 4F) is exactly on the generalized-lune boundary of i = (0, 0),
    j = (6F, 8F) with r_i = 2F, r_j = F, so (i, j) stays linked; moving k by
    one grid unit inward breaks the link."""
    say("grng exact ties")
    F = 2 ** 20
    from oracle import grng as ogr
    for k in ([3 * F, 4 * F], [3 * F, 4 * F - 1], [3 * F + 1, 4 * F]):
        P = np.array([[0, 0], [6 * F, 8 * F], k, [12 * F, 0], [0, 9 * F]], np.float32)
        R = np.array([2 * F, F, 0, F, 3], np.float32)
        want = ogr.grng_edges(exact.to_grid(P, 0), R.astype(np.int64))
        idx = G.Index(to_dev(P), grid_exp=0)
        idx.build_grng_layer(0, to_dev(np.arange(5, dtype=np.int32)), to_dev(R))
        got = idx.edges(0).cpu().numpy().astype(np.int64)
        st = idx.stats()
        idx.close()
        assert np.array_equal(got, want), k
        if k == [3 * F, 4 * F]:
            assert st["rechecks"] > 0


@pytest.mark.parametrize("n,d,mf,mc,seed,prec", [(6000, 32, 240, 12, 0, 0), (6000, 32, 240, 12, 0, 1),
                                                 (6000, 32, 240, 12, 0, 2), (3000, 8, 150, 20, 1, 1),
                                                 (3000, 8, 150, 20, 1, 2)])
def test_three_layer_hierarchy_matches_oracle(G, n, d, mf, mc, seed, prec):
    """Coarse layer -> guided fine layer (Theorem 2) -> RNG, on the
    8-dimensional-subspace workload family at reduced size."""
    say("three layers", n, d, mf, mc, seed, "precision", prec)
    W = synth.subspace3(n=n, d=d, m_fine=mf, m_coarse=mc, sub=seed)
    (Lc, Lf) = W.layers
    E, lay, st = gpu_edges(G, W.X, W.q, [(Lc.pivot_ids, Lc.radii), (Lf.pivot_ids, Lf.radii)], precision=prec)
    assert np.array_equal(lay[0], Lc.pivot_ids[native.grng_edges(W.X[Lc.pivot_ids], Lc.radii, W.q)])
    assert np.array_equal(lay[1], Lf.pivot_ids[native.grng_edges(W.X[Lf.pivot_ids], Lf.radii, W.q)])
    assert np.array_equal(E, native.rng_edges(W.X, W.q))


def test_failed_allocation_leaves_the_index_unchanged(G, monkeypatch):
    """GRNG_FAIL_ALLOC_AT=k fails the k-th device allocation of a call: the
    call returns ENOMEM and the index keeps its previous graph, so later calls
    work as before."""
    say("failure injection in build_rng and insert_batch")
    W = synth.clustered(n=3000, d=16, clusters=8, m=60, knn=40)
    L = W.layers[0]
    idx = G.Index(to_dev(W.X), grid_exp=W.q, precision=1)
    idx.build_grng_layer(0, to_dev(L.pivot_ids), to_dev(L.radii))
    idx.build_rng()
    E0 = idx.edges().cpu().numpy()
    B = synth.insert_batches(W, n_batches=1, lo=300, hi=301, sub=9)[0]
    for k in (1, 5, 20):
        monkeypatch.setenv("GRNG_FAIL_ALLOC_AT", str(k))
        with pytest.raises(G.GrngError) as e:
            idx.build_rng()
        assert e.value.status == -2, k
        with pytest.raises(G.GrngError) as e:
            idx.insert_batch(to_dev(B))
        assert e.value.status == -2, k
        monkeypatch.delenv("GRNG_FAIL_ALLOC_AT")
        assert np.array_equal(idx.edges().cpu().numpy(), E0), k
        assert idx.stats()["n_points"] == W.n
    idx.build_rng()
    assert np.array_equal(idx.edges().cpu().numpy(), E0)
    idx.insert_batch(to_dev(B))
    E1 = idx.edges().cpu().numpy()
    assert np.array_equal(E1.astype(np.int64), native.rng_edges(np.vstack([W.X, B]), W.q))
    # A second, smaller batch fits the room the first insertion left in the
    # kept distance table, so the insertion hands that table to the new state
    # and must give it back when a later allocation fails.
    B2 = synth.insert_batches(W, n_batches=1, lo=100, hi=101, sub=10)[0]
    failed = 0
    for k in (1, 10, 30, 50, 70, 90, 120, 160, 220, 300, 400, 600):
        monkeypatch.setenv("GRNG_FAIL_ALLOC_AT", str(k))
        try:
            idx.insert_batch(to_dev(B2))
        except G.GrngError as e:
            assert e.status == -2, k
            failed += 1
            monkeypatch.delenv("GRNG_FAIL_ALLOC_AT")
            assert np.array_equal(idx.edges().cpu().numpy(), E1), k
            assert idx.stats()["n_points"] == W.n + len(B), k
            continue
        monkeypatch.delenv("GRNG_FAIL_ALLOC_AT")
        break   # fewer than k allocations: the insertion went through
    say("insertion failed at", failed, "allocation counts before it went through")
    assert failed >= 4
    if idx.stats()["n_points"] == W.n + len(B):
        idx.insert_batch(to_dev(B2))
    assert np.array_equal(idx.edges().cpu().numpy().astype(np.int64),
                          native.rng_edges(np.vstack([W.X, B, B2]), W.q))
    idx.close()


_FOUR_LAYER_ORACLE = {}


@pytest.mark.parametrize("ms,prec", [((10, 60, 400), 1), ((10, 60, 400), 2), ((6, 40, 200), 0)])
def test_four_layer_hierarchy_matches_oracle(G, ms, prec):
    """Three nested pivot layers over the exemplars (a four-layer hierarchy):
    each finer layer guided by the one above it (Section 3, Theorem 2), the
    RNG guided by the finest; every layer and the RNG equal the oracle's."""
    say("four-layer hierarchy n=12000 d=32 layers", ms, "precision", prec)
    W = synth.subspace_layers(12000, ms=ms)
    for coarse, fine in zip(W.layers, W.layers[1:]):
        assert set(coarse.pivot_ids) <= set(fine.pivot_ids)
    E, lay, st = gpu_edges(G, W.X, W.q, [(L.pivot_ids, L.radii) for L in W.layers], precision=prec)
    assert st["n_layers"] == 3
    for l, L in enumerate(W.layers):
        assert np.array_equal(lay[l], L.pivot_ids[native.grng_edges(W.X[L.pivot_ids], L.radii, W.q)]), l
    if ms not in _FOUR_LAYER_ORACLE:
        _FOUR_LAYER_ORACLE[ms] = native.rng_edges(W.X, W.q)
    assert np.array_equal(E, _FOUR_LAYER_ORACLE[ms])
