"""The allocation-free gradient entry point against the allocating one (needs an MI355X).

grng_mlp_grad_noalloc keeps its per-block partial gradients in the library's
fixed device scratch instead of allocating them; it runs the same kernels in
the same block decomposition, so its loss and gradient must equal
grng_mlp_grad's bit for bit.  Two calls in a row, the second with fewer
samples (it must not read partials left by the first).
"""
import ctypes as C

import numpy as np
import pytest
from conftest import say

pytestmark = pytest.mark.gpu


def _inputs(n, seed):
    import torch
    import paper_2208_10022_amd as P
    g = np.random.default_rng(seed)
    feats = torch.from_numpy(g.standard_normal((n, P.MLP_FEATURES)).astype(np.float32)).cuda()
    labels = torch.from_numpy((g.random(n) < 0.3).astype(np.uint8)).cuda()
    return feats, labels


def test_noalloc_gradient_equals_the_allocating_one():
    import torch
    import paper_2208_10022_amd as P
    assert torch.cuda.is_available()
    g = np.random.default_rng(1)
    theta = torch.from_numpy((0.2 * g.standard_normal(P.mlp_params())).astype(np.float32)).cuda()
    grad = torch.empty(P.mlp_params(), dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    for n, seed in ((300_000, 2), (5_000, 3)):
        say("noalloc gradient n", n)
        feats, labels = _inputs(n, seed)
        want_g, want_l = P.mlp_grad(theta, feats, labels)
        P.mlp_grad_noalloc(theta, feats, labels, grad, loss)
        torch.cuda.synchronize()
        assert torch.equal(grad, want_g), n
        assert float(loss.item()) == want_l, n
    # sizes beyond the fixed scratch are refused before any launch
    lib = P.lib()
    st = lib.grng_mlp_grad_noalloc(C.c_void_p(theta.data_ptr()), C.c_void_p(feats.data_ptr()),
                                   C.c_void_p(labels.data_ptr()), P.MLP_NOALLOC_MAX_SAMPLES + 1,
                                   C.c_void_p(grad.data_ptr()), C.c_void_p(loss.data_ptr()), None)
    assert st == -1
    st = lib.grng_mlp_grad_noalloc(C.c_void_p(theta.data_ptr()), C.c_void_p(feats.data_ptr()),
                                   C.c_void_p(labels.data_ptr()), 0, C.c_void_p(grad.data_ptr()),
                                   C.c_void_p(loss.data_ptr()), None)
    assert st == -1
