"""GPU checks of the learned witness-domain ranking (needs an MI355X).

The gradient, Adam step and bf16 scoring kernels are compared with the
float64 reference in oracle/mlp.py; the learned visit order must leave every
edge unchanged (integer output: bit-exact against the oracle's edges).
"""
import os

import numpy as np
import pytest

import synth
from oracle import mlp, native
from conftest import say

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
F, H = 9, 64   # features, hidden units of the library's scorer


@pytest.fixture(scope="module")
def G():
    import torch
    import paper_2208_10022_amd as P
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    P.lib()
    assert P.mlp_params() == F * H + 2 * H + 1
    return P


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _data(seed, n):
    g = np.random.default_rng(seed)
    theta = (g.standard_normal(F * H + 2 * H + 1) * 0.3).astype(np.float32)
    X = (g.standard_normal((n, F)) * 1.5).astype(np.float32)
    y = (g.random(n) < 0.3).astype(np.uint8)
    return theta, X, y


@pytest.mark.parametrize("n", [1, 63, 64, 4096, 10001])
def test_gradient_matches_float64_backprop(G, n):
    # 10001 spans three 4096-sample blocks and a ragged last LDS batch.
    say("mlp grad n=%d" % n)
    theta, X, y = _data(n, n)
    g, loss = G.mlp_grad(to_dev(theta), to_dev(X), to_dev(y))
    want = mlp.grad(theta.astype(np.float64), X.astype(np.float64), y, F, H)
    got = g.cpu().numpy().astype(np.float64)
    # float32 sums of n terms: error well below 1e-4 of the largest component.
    scale = np.abs(want).max()
    assert np.allclose(got, want, rtol=1e-3, atol=1e-4 * scale), np.abs(got - want).max() / scale
    assert abs(loss - mlp.loss(theta, X, y, F, H)) <= 1e-5 * max(1.0, abs(loss))


def test_adam_step_matches_reference(G):
    say("mlp adam, one step")
    theta, X, y = _data(5, 3000)
    lr = 1e-3
    t = to_dev(theta.copy())
    G.mlp_train(t, to_dev(X), to_dev(y), steps=1, lr=lr)
    g64 = mlp.grad(theta.astype(np.float64), X.astype(np.float64), y, F, H)
    want, _, _ = mlp.adam_step(theta.astype(np.float64), g64, np.zeros_like(g64), np.zeros_like(g64), 1, lr)
    got = t.cpu().numpy().astype(np.float64)
    # A first Adam step moves each parameter by lr * g / (|g| + eps): where
    # the gradient is far from zero both sides move by lr in the same
    # direction; near zero the float32 gradient may differ in sign.
    firm = np.abs(g64) > 1e-3 * np.abs(g64).max()
    assert firm.sum() > 0.5 * firm.size
    assert np.allclose(got[firm], want[firm], rtol=0, atol=1e-6)
    assert np.all(np.abs(got - theta) <= lr * (1 + 1e-4))


def test_training_lowers_loss(G):
    say("mlp train 200 steps")
    theta, X, _ = _data(9, 20000)
    # labels from a fixed rule the network can learn
    y = ((X[:, 0] - 0.5 * X[:, 3]) < 0.2).astype(np.uint8)
    t = to_dev(theta)
    l0 = G.mlp_grad(t, to_dev(X), to_dev(y))[1]
    l1 = G.mlp_train(t, to_dev(X), to_dev(y), steps=200, lr=1e-2)
    assert l1 < 0.5 * l0
    assert abs(l1 - mlp.loss(t.cpu().numpy(), X, y, F, H)) <= 1e-4


@pytest.mark.parametrize("n", [0, 1, 257])
def test_scores_use_bf16_weights(G, n):
    say("mlp score n=%d" % n)
    theta, X, _ = _data(11, max(n, 1))
    X = X[:n]
    s = G.mlp_score(to_dev(theta), to_dev(X)).cpu().numpy().astype(np.float64)
    assert s.shape == (n,)
    if n == 0:
        return
    want = mlp.forward(mlp.bf16_round(theta), X.astype(np.float64), F, H)
    ref_scale = np.abs(mlp.forward(np.abs(mlp.bf16_round(theta)), np.abs(X.astype(np.float64)), F, H))
    # float32 accumulation of ~600 products: a few ulps of the magnitude sum
    assert np.all(np.abs(s - want) <= 1e-5 * ref_scale + 1e-6)
    # and the scores are not the float32-weight ones (the rounding is real)
    exact = mlp.forward(theta.astype(np.float64), X.astype(np.float64), F, H)
    assert np.abs(exact - want).max() > 0


def _clustered_small():
    return synth.clustered(n=3000, d=16, clusters=8, m=60, knn=40)


def _golden(name):
    rows = [ln.split() for ln in open(os.path.join(HERE, "golden", name)) if ln.strip() and not ln.startswith("#")]
    return np.array(rows, dtype=np.int64).reshape(-1, 2)


def _build(G, W, theta=None, precision=0, **kw):
    # precision 0: both orders run the per-pair exhaustive scan, so their
    # witness-test counts compare like with like
    L = W.layers[0]
    idx = G.Index(to_dev(W.X), grid_exp=W.q, witness_order=G.ORDER_LEARNED if theta is not None else 0,
                  precision=precision, **kw)
    idx.build_grng_layer(0, to_dev(L.pivot_ids), to_dev(L.radii))
    if theta is not None:
        idx.set_scorer(theta)
    idx.build_rng()
    return idx


def test_learned_order_needs_a_scorer(G):
    say("learned order without scorer")
    W = _clustered_small()
    L = W.layers[0]
    idx = G.Index(to_dev(W.X), grid_exp=W.q, witness_order=G.ORDER_LEARNED)
    idx.build_grng_layer(0, to_dev(L.pivot_ids), to_dev(L.radii))
    with pytest.raises(G.GrngError) as e:
        idx.build_rng()
    assert e.value.status == -6
    with pytest.raises(G.GrngError) as e:
        idx.log_witness_cells(10)
    assert e.value.status == -6
    idx.close()


def test_logged_samples_are_well_formed(G):
    say("log witness cells, clustered n=3000")
    W = _clustered_small()
    idx = _build(G, W)
    st = idx.stats()
    feats, labels = idx.log_witness_cells(500)
    f = feats.cpu().numpy()
    lab = labels.cpu().numpy()
    assert f.shape[0] == lab.shape[0] > 0
    assert set(np.unique(lab)) <= {0, 1}
    assert np.all(np.isfinite(f)) and np.all(np.abs(f) <= 64)
    # every logged domain passed Proposition 3 (margin feature below 1)
    assert np.all(f[:, 4] < 1.0)
    # the smaller and the larger of the two relative pivot distances (the
    # larger is the lune-order key); rounding and clipping are monotone
    assert np.array_equal(f[:, 7], np.minimum(f[:, 0], f[:, 1]))
    assert np.array_equal(f[:, 8], np.maximum(f[:, 0], f[:, 1]))
    assert st["exhaustive_pairs"] > 0
    # the sample list is the same on every call (training is reproducible)
    f2, lab2 = idx.log_witness_cells(500)
    assert np.array_equal(f2.cpu().numpy(), f) and np.array_equal(lab2.cpu().numpy(), lab)
    # labels are exact: some domains hold witnesses, some do not
    assert 0 < lab.sum() < len(lab)
    idx.close()


def _train_scorer(G, idx, steps=300):
    import torch
    feats, labels = idx.log_witness_cells(4000)
    theta = torch.from_numpy((np.random.default_rng(1).standard_normal(F * H + 2 * H + 1) * 0.1)
                             .astype(np.float32)).cuda()
    l0 = G.mlp_grad(theta, feats, labels)[1]
    l1 = G.mlp_train(theta, feats, labels, steps=steps, lr=3e-3)
    return theta, l0, l1


def test_learned_order_keeps_edges_identical(G):
    say("learned order, clustered n=3000 vs golden")
    W = _clustered_small()
    base = _build(G, W)
    theta, l0, l1 = _train_scorer(G, base)
    assert l1 < l0
    st0 = base.stats()
    base.close()
    idx = _build(G, W, theta)
    E = idx.edges().cpu().numpy().astype(np.int64)
    st1 = idx.stats()
    assert np.array_equal(E, _golden("clustered_n3000_d16_rng_edges.txt"))
    say("witness tests distance order %d, learned %d" % (st0["witness_tests"], st1["witness_tests"]))
    # queries and insertions take the same scan: results equal the oracle's
    g = np.random.default_rng(4)
    Q = synth.queries_like(W, 40, sub=1)
    off, nb = idx.query_neighbors(to_dev(Q))
    off = off.cpu().numpy()
    nb = nb.cpu().numpy()
    for i in g.choice(len(Q), 8, replace=False):
        want = native.query_row(W.X, W.q, Q[i])
        assert np.array_equal(np.sort(nb[off[i]:off[i + 1]]), np.sort(want))
    # a random scorer also keeps the edges
    rnd = to_dev((np.random.default_rng(2).standard_normal(F * H + 2 * H + 1)).astype(np.float32))
    idx.set_scorer(rnd)
    idx.build_rng()
    assert np.array_equal(idx.edges().cpu().numpy().astype(np.int64), E)
    idx.close()


def test_learned_order_gain_at_scale(G):
    """Witness tests with the trained order vs the distance order (same edges)."""
    W = synth.clustered(n=30000, d=16, clusters=32, m=300, knn=100)
    say("learned order gain, clustered n=30000 m=300")
    base = _build(G, W)
    E0 = base.edges().cpu().numpy()
    st0 = base.stats()
    theta, l0, l1 = _train_scorer(G, base, steps=400)
    base.close()
    idx = _build(G, W, theta)
    st1 = idx.stats()
    assert np.array_equal(idx.edges().cpu().numpy(), E0)
    say("loss %.4f -> %.4f; exhaustive witness tests: distance %d, learned %d (%.3fx)"
        % (l0, l1, st0["lune_tests"], st1["lune_tests"], st0["lune_tests"] / max(st1["lune_tests"], 1)))
    assert l1 < l0
    # the trained order spends fewer witness tests than the distance order
    assert st1["lune_tests"] < st0["lune_tests"]
    idx.close()
