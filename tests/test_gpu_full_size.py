"""Parity at the full size of every workload (needs an MI355X).

* 100k x 16-D, 1,000 pivots: the complete RNG edge set of every arithmetic
  form equals the oracle's (count and sha256 of the canonical array, written
  by tests/golden/make_golden.py from the C oracle); the pivot GRNG in full.
* 1M x 32-D, 100 / 3,000 pivots: the bf16 and float32 forms give the same
  complete edge set; both GRNG layers in full; 1,000+ RNG rows against the
  oracle.
* 64 insertion batches into the 100k index: after every batch the complete
  edge set equals a rebuild from scratch of all points so far (a different
  code path); 1,000+ oracle rows over the run, most of them points of the
  batches and endpoints of edges the batches removed.
* 1M x 96-D, 10,000 pivots: the distance-order and learned-order scans give
  the same complete edge set; 1,000+ oracle rows.

Oracle rows are not sampled uniformly only: they include orphans (points in
no pivot domain), members of the largest home cells, endpoints of the
longest edges and the highest-degree points.  They are computed on the host
in a background thread while the GPU builds (the C oracle releases the GIL).
"""
import hashlib
import os
import threading

import numpy as np
import pytest

import synth
from oracle import native
from conftest import say

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def G():
    import torch
    import paper_2208_10022_amd as P
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    P.lib()
    native.build(force=False)
    return P


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


class OracleRows(threading.Thread):
    """RNG rows of the points xs by the C oracle, on the host, in the background."""

    def __init__(self, X, q, xs):
        super().__init__(daemon=True)
        self.X, self.q, self.xs = X, q, np.asarray(xs, dtype=np.int64)
        self.rows, self.error = None, None
        self.start()

    def run(self):
        try:
            self.rows = native.rng_rows_compact(self.X, self.q, self.xs)
        except BaseException as e:   # re-raised in the test thread
            self.error = e

    def get(self):
        self.join()
        if self.error is not None:
            raise self.error
        return self.rows


def neighbour_lists(E, xs):
    """Neighbours of each x in xs from a canonical edge array (u < v)."""
    both = np.concatenate([E, E[:, ::-1]])
    both = both[np.argsort(both[:, 0], kind="stable")]
    lo = np.searchsorted(both[:, 0], xs, side="left")
    hi = np.searchsorted(both[:, 0], xs, side="right")
    return [np.sort(both[a:b, 1]) for a, b in zip(lo, hi)]


def check_rows(E, xs, want, what):
    got = neighbour_lists(E, xs)
    bad = [int(x) for x, g, w in zip(xs, got, want) if not np.array_equal(g, w)]
    assert not bad, "%s: %d of %d rows differ, e.g. %s" % (what, len(bad), len(xs), bad[:5])
    say("%s: %d oracle rows equal" % (what, len(xs)))


def pivot_cells(X, pid, rad):
    """Home cell (nearest pivot) and orphan flag (in no pivot ball) of every
    point, on the GPU in float64 (exact on the grid); used only to choose
    which rows to check."""
    import torch
    Xd = torch.from_numpy(X).cuda().double()
    P = Xd[torch.from_numpy(pid.astype(np.int64)).cuda()]
    r2 = torch.from_numpy(rad.astype(np.float64)).cuda() ** 2
    pn = (P * P).sum(1)
    home = torch.empty(len(X), dtype=torch.int64, device="cuda")
    orphan = torch.empty(len(X), dtype=torch.bool, device="cuda")
    for s in range(0, len(X), 1 << 16):
        x = Xd[s:s + (1 << 16)]
        d2 = (x * x).sum(1, keepdim=True) + pn[None, :] - 2.0 * (x @ P.T)
        home[s:s + len(x)] = d2.argmin(1)
        orphan[s:s + len(x)] = ~(d2 <= r2[None, :]).any(1)
    return home.cpu().numpy(), orphan.cpu().numpy()


def pick_rows(X, E, layer, n_random, seed, extra=()):
    """About n_random random rows plus targeted ones (see the module docstring)."""
    g = np.random.default_rng(seed)
    n = len(X)
    picks = [g.choice(n, n_random, replace=False), np.asarray(extra, dtype=np.int64)]
    home, orphan = pivot_cells(X, layer.pivot_ids, layer.radii)
    orph = np.nonzero(orphan)[0]
    if len(orph):
        picks.append(g.choice(orph, min(100, len(orph)), replace=False))
    big = np.argsort(np.bincount(home, minlength=len(layer.pivot_ids)))[-5:]
    for c in big:
        mem = np.nonzero(home == c)[0]
        picks.append(g.choice(mem, min(20, len(mem)), replace=False))
    if len(E):
        L = ((X[E[:, 0]].astype(np.float64) - X[E[:, 1]].astype(np.float64)) ** 2).sum(1)
        picks.append(E[np.argsort(L)[-50:]].reshape(-1))
        deg = np.bincount(E.reshape(-1), minlength=n)
        picks.append(np.argsort(deg)[-50:])
    return np.unique(np.concatenate(picks))


def build(G, W, layers, **kw):
    idx = G.Index(to_dev(W.X), grid_exp=W.q, **kw)
    for l, L in enumerate(layers):
        idx.build_grng_layer(l, to_dev(L.pivot_ids), to_dev(L.radii))
    return idx


def edges_and_close(idx, nlayers):
    idx.build_rng()
    E = idx.edges().cpu().numpy().astype(np.int64)
    lay = [idx.edges(l).cpu().numpy().astype(np.int64) for l in range(nlayers)]
    st = idx.stats()
    idx.close()
    return E, lay, st


def digest(E):
    A = np.ascontiguousarray(np.asarray(E, dtype="<i4").reshape(-1, 2))
    return len(A), hashlib.sha256(A.tobytes()).hexdigest()


def golden_digest(name):
    vals = {}
    for ln in open(os.path.join(HERE, "golden", name)):
        if ln.strip() and not ln.startswith("#"):
            k, v = ln.split()
            vals[k] = v
    return int(vals["edges"]), vals["sha256"]


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_clustered_full_size_complete_edge_set(G, prec):
    """The complete RNG of the 100k x 16-D workload equals the oracle's, in
    every arithmetic form; the 1,000-pivot GRNG in full."""
    say("clustered full size n=100000 d=16 m=1000, complete edge set, precision", prec)
    W = synth.clustered()
    L = W.layers[0]
    E, lay, st = edges_and_close(build(G, W, W.layers, precision=prec), 1)
    say("stats", {k: st[k] for k in ("n_edges", "exhaustive_pairs", "rechecks", "screen_uncertain", "ms_rng")})
    assert digest(E) == golden_digest("clustered_n100000_d16_rng_digest.txt")
    assert np.array_equal(lay[0], L.pivot_ids[native.grng_edges(W.X[L.pivot_ids], L.radii, W.q)])


def test_subspace3_full_size_forms_and_oracle_rows(G):
    """1M x 32-D near an 8-D subspace, 100 coarse / 3,000 fine pivots: the
    bf16 form (the workload's) and the float32 form give the same complete
    edge set; both layers equal the oracle's in full; 1,000+ oracle rows."""
    say("subspace3 full size n=1000000 d=32 m=100/3000")
    W = synth.subspace3()
    Lc, Lf = W.layers
    E2, lay, st2 = edges_and_close(build(G, W, W.layers, precision=2), 2)
    say("bf16 stats", {k: st2[k] for k in ("n_edges", "exhaustive_pairs", "screen_uncertain", "ms_rng")})
    rows = pick_rows(W.X, E2, Lf, 800, 7)
    orc = OracleRows(W.X, W.q, rows)
    E1, lay1, st1 = edges_and_close(build(G, W, W.layers, precision=1), 2)
    say("float32 stats", {k: st1[k] for k in ("n_edges", "exhaustive_pairs", "rechecks", "ms_rng")})
    assert np.array_equal(E1, E2)
    assert np.array_equal(lay1[0], lay[0]) and np.array_equal(lay1[1], lay[1])
    assert np.array_equal(lay[0], Lc.pivot_ids[native.grng_edges(W.X[Lc.pivot_ids], Lc.radii, W.q)])
    assert np.array_equal(lay[1], Lf.pivot_ids[native.grng_edges(W.X[Lf.pivot_ids], Lf.radii, W.q)])
    assert len(rows) >= 1000
    check_rows(E2, rows, orc.get(), "subspace3")


def test_insert_64_batches_each_equals_a_rebuild(G):
    """Config 4: 64 batches of log-uniform sizes in [1,000, 50,000] into the
    100k x 16-D index.  After every batch the complete edge set equals a
    rebuild from scratch of all points so far; oracle rows of batch points,
    of endpoints of removed edges, orphans and random points."""
    say("insert 64 batches into the 100k index, rebuild after each")
    W = synth.clustered()
    L = W.layers[0]
    batches = synth.insert_batches(W)
    idx = build(G, W, W.layers, precision=1)
    idx.build_rng()
    E_prev = idx.edges().cpu().numpy().astype(np.int64)
    allX = [W.X]
    g = np.random.default_rng(11)
    pending = []
    checked = 0
    for bi, B in enumerate(batches, 1):
        idx.insert_batch(to_dev(B))
        allX.append(B)
        X = np.vstack(allX)
        E = idx.edges().cpu().numpy().astype(np.int64)
        Wb = synth.Workload(name="insert", X=X, q=W.q)
        Er, _, _ = edges_and_close(build(G, Wb, W.layers, precision=1), 1)
        assert np.array_equal(E, Er), bi
        say("batch", bi, "of", len(batches), "n", len(X), "equals the rebuild")
        if bi in (1, 2, 8, 16, 32, 64):
            n0 = len(X) - len(B)
            prev = {(int(u), int(v)) for u, v in E_prev}
            now = {(int(u), int(v)) for u, v in E}
            removed = np.array(sorted(prev - now), dtype=np.int64).reshape(-1, 2)
            extra = [n0 + g.choice(len(B), min(60, len(B)), replace=False)]
            if len(removed):
                extra.append(removed[g.choice(len(removed), min(30, len(removed)), replace=False)].reshape(-1))
            rows = pick_rows(X, E, L, 40, bi, np.concatenate(extra))
            pending.append((bi, E, rows, OracleRows(X, W.q, rows)))
            checked += len(rows)
            say("batch", bi, "n", len(X), "edges", len(E), "removed", len(removed), "rows", len(rows))
        E_prev = E
    idx.close()
    assert checked >= 1000
    for bi, E, rows, orc in pending:
        check_rows(E, rows, orc.get(), "after batch %d" % bi)


def _scorer_from_clustered16(G):
    """Scorer trained on logged witness cells of the 100k x 16-D build and of
    a small 2-D build (the training set the learned form is specified with)."""
    import torch
    feats, labels = [], []
    for W in (synth.clustered(), synth.clustered(n=20000, d=2, clusters=16, m=200, knn=50, q=19, sub=3)):
        idx = build(G, W, W.layers, precision=1)
        idx.build_rng()
        f, lab = idx.log_witness_cells(20000)
        feats.append(f)
        labels.append(lab)
        idx.close()
    feats, labels = torch.cat(feats), torch.cat(labels)
    theta = torch.from_numpy((np.random.default_rng(1).standard_normal(G.mlp_params()) * 0.1)
                             .astype(np.float32)).cuda()
    l0 = G.mlp_grad(theta, feats, labels)[1]
    l1 = G.mlp_train(theta, feats, labels, steps=400, lr=3e-3)
    assert l1 < l0
    return theta


def test_clustered96_full_size_orders_and_oracle_rows(G):
    """1M x 96-D, 256 clusters, 10,000 pivots: the learned and lune-key visit
    orders give the same complete edge set as the distance order; 1,000+
    oracle rows."""
    say("clustered96 full size n=1000000 d=96 m=10000")
    theta = _scorer_from_clustered16(G)
    W = synth.clustered(n=1_000_000, d=96, clusters=256, sigma=1.0, m=10_000, knn=100, q=18)
    L = W.layers[0]
    idx = build(G, W, W.layers, precision=1, witness_order=G.ORDER_LEARNED)
    idx.set_scorer(theta)
    E_l, _, st_l = edges_and_close(idx, 1)
    say("learned stats", {k: st_l[k] for k in ("n_edges", "lune_tests", "ms_lune", "ms_rng")})
    rows = pick_rows(W.X, E_l, L, 800, 9)
    orc = OracleRows(W.X, W.q, rows)
    E_d, _, st_d = edges_and_close(build(G, W, W.layers, precision=1), 1)
    say("distance-order stats", {k: st_d[k] for k in ("n_edges", "lune_tests", "ms_lune", "ms_rng")})
    assert np.array_equal(E_d, E_l)
    E_k, _, st_k = edges_and_close(build(G, W, W.layers, precision=1, witness_order=G.ORDER_LUNE), 1)
    say("lune-key-order stats", {k: st_k[k] for k in ("n_edges", "lune_tests", "ms_lune", "ms_rng")})
    assert np.array_equal(E_d, E_k)
    assert len(rows) >= 1000
    check_rows(E_d, rows, orc.get(), "clustered96")
