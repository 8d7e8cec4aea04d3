"""Python binding of the gfx950 exact RNG / GRNG library ``libgrng.so``.

Argument marshalling only: every step of the build runs in the library's HIP
kernels.  PyTorch supplies device memory (tensor data pointers) and the
current HIP stream; nothing here computes distances, lunes or edges.  The
names follow the C ABI in ``include/grng.h``.  If the library is missing this
module raises at load time: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgrng.so")

GRNG_OK, GRNG_ECAPACITY = 0, -5
STATUS_NAMES = {0: "GRNG_OK", -1: "GRNG_EINVAL", -2: "GRNG_ENOMEM", -3: "GRNG_EDEVICE", -4: "GRNG_ENOTGRID",
                -5: "GRNG_ECAPACITY", -6: "GRNG_ESTATE"}
PREC_FP64, PREC_FP32, PREC_BF16, PREC_AUTO = 0, 1, 2, 3
ORDER_DISTANCE, ORDER_LEARNED, ORDER_LUNE = 0, 1, 2
METRIC_L2, METRIC_L1, METRIC_LINF = 0, 1, 2
GRAPH_RNG, GRAPH_GABRIEL, GRAPH_BETA = 0, 1, 2

# Entry points declared in include/grng.h (checked by the CPU tests).
ABI_FUNCTIONS = ("grng_abi_version", "grng_last_error", "grng_create", "grng_build_grng_layer", "grng_build_rng",
                 "grng_insert_batch", "grng_query_neighbors", "grng_get_edges", "grng_get_stats", "grng_destroy",
                 "grng_mlp_params", "grng_mlp_grad", "grng_mlp_grad_noalloc", "grng_mlp_train", "grng_mlp_score", "grng_log_witness_cells",
                 "grng_set_scorer", "grng_insert_pivots", "grng_get_orphans")
MLP_FEATURES, MLP_HIDDEN = 9, 64


class GrngError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, str(status)), message))
        self.status = status


class Options(C.Structure):
    _fields_ = [("grid_exp", C.c_int32), ("precision", C.c_int32), ("witness_order", C.c_int32),
                ("use_graph", C.c_int32), ("autotune", C.c_int32), ("stage4_pivots", C.c_int32),
                ("vgrng_pivots", C.c_int32), ("metric", C.c_int32), ("graph", C.c_int32),
                ("beta_quarters", C.c_int32), ("reserved", C.c_uint64 * 3)]


class Stats(C.Structure):
    _fields_ = [("n_points", C.c_int64), ("n_edges", C.c_int64), ("n_layers", C.c_int64), ("orphans", C.c_int64),
                ("tile_pairs", C.c_int64), ("vgrng_pivots", C.c_int64), ("stage4_pivots", C.c_int64),
                ("unsorted_cell_rows", C.c_int64),
                ("distance_computations", C.c_double), ("witness_tests", C.c_double),
                ("candidate_pairs", C.c_double), ("stage4_survivors", C.c_double),
                ("exhaustive_pairs", C.c_double), ("lune_tests", C.c_double), ("rechecks", C.c_double),
                ("ms_layers", C.c_double), ("ms_rng", C.c_double), ("ms_insert", C.c_double),
                ("ms_query", C.c_double), ("ms_vgrng", C.c_double), ("ms_pairs", C.c_double),
                ("ms_lune", C.c_double), ("vgrng_ops", C.c_double), ("pairs_flops", C.c_double),
                ("lune_bytes", C.c_double), ("stage4_ops", C.c_double), ("ms_autotune", C.c_double),
                ("ms_pair_masks", C.c_double), ("screen_uncertain", C.c_double),
                ("pair_tile_entries", C.c_double), ("pair_method_distances", C.c_double),
                ("lune_tests_kept", C.c_double), ("partner_tests", C.c_double), ("partner_kills", C.c_double),
                ("ms_partner", C.c_double), ("precision_used", C.c_int64)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_ if not name.startswith("reserved")}


_lib = None


def lib():
    """Load libgrng.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libgrng.so is not built; run paper_2208_10022_amd/build.py "
                              "(or __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
        sig = {
            "grng_abi_version": (i32, []),
            "grng_last_error": (C.c_char_p, []),
            "grng_create": (i32, [C.POINTER(vp), vp, i64, i32, vp, C.POINTER(Options)]),
            "grng_build_grng_layer": (i32, [vp, i32, vp, vp, i64]),
            "grng_build_rng": (i32, [vp]),
            "grng_insert_batch": (i32, [vp, vp, i64]),
            "grng_insert_pivots": (i32, [vp, i32, vp, vp, i64]),
            "grng_get_orphans": (i32, [vp, vp, i64, C.POINTER(i64)]),
            "grng_query_neighbors": (i32, [vp, vp, i64, vp, vp, i64, C.POINTER(i64)]),
            "grng_get_edges": (i32, [vp, i32, vp, i64, C.POINTER(i64)]),
            "grng_get_stats": (i32, [vp, C.POINTER(Stats)]),
            "grng_destroy": (None, [vp]),
            "grng_mlp_params": (i32, []),
            "grng_mlp_grad": (i32, [vp, vp, vp, i64, vp, C.POINTER(C.c_float), vp]),
            "grng_mlp_grad_noalloc": (i32, [vp, vp, vp, i64, vp, vp, vp]),
            "grng_mlp_train": (i32, [vp, vp, vp, i64, i32, C.c_float, C.POINTER(C.c_float), vp]),
            "grng_mlp_score": (i32, [vp, vp, i64, vp, vp]),
            "grng_log_witness_cells": (i32, [vp, i64, vp, vp, i64, C.POINTER(i64)]),
            "grng_set_scorer": (i32, [vp, vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().grng_last_error().decode()


def check(status: int) -> None:
    if status != GRNG_OK:
        raise GrngError(status, last_error())


def _dev_ptr(t, dtype_name: str, ndim: int | None = None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a device tensor")
    if str(t.dtype) != "torch." + dtype_name:
        raise TypeError("expected dtype %s, got %s" % (dtype_name, t.dtype))
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if ndim is not None and t.dim() != ndim:
        raise ValueError("expected %d dimensions" % ndim)
    return C.c_void_p(t.data_ptr())


def _stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def mlp_params() -> int:
    return int(lib().grng_mlp_params())


def _mlp_inputs(theta, feats, labels=None):
    if theta.numel() != mlp_params():
        raise ValueError("theta must hold %d parameters" % mlp_params())
    if feats.dim() != 2 or feats.shape[1] != MLP_FEATURES:
        raise ValueError("feats must be [n, %d]" % MLP_FEATURES)
    if labels is not None and labels.numel() != feats.shape[0]:
        raise ValueError("one label per feature row")


def mlp_grad(theta, feats, labels, stream=None):
    """(gradient float32 [P] device tensor, loss) of the witness-domain scorer."""
    import torch
    _mlp_inputs(theta, feats, labels)
    g = torch.empty_like(theta)
    loss = C.c_float(0.0)
    check(lib().grng_mlp_grad(_dev_ptr(theta, "float32"), _dev_ptr(feats, "float32"), _dev_ptr(labels, "uint8"),
                              feats.shape[0], _dev_ptr(g, "float32"), C.byref(loss), _stream_handle(stream)))
    return g, float(loss.value)


MLP_NOALLOC_MAX_SAMPLES = 1 << 24


def mlp_grad_noalloc(theta, feats, labels, grad_out, loss_out, stream=None) -> None:
    """grng_mlp_grad_noalloc: gradient into grad_out (float32 [P], device) and the
    loss into loss_out (float32 [1], device); the library allocates nothing."""
    _mlp_inputs(theta, feats, labels)
    if grad_out.numel() != mlp_params() or loss_out.numel() < 1:
        raise ValueError("grad_out must hold %d floats and loss_out at least one" % mlp_params())
    check(lib().grng_mlp_grad_noalloc(_dev_ptr(theta, "float32"), _dev_ptr(feats, "float32"),
                                      _dev_ptr(labels, "uint8"), feats.shape[0], _dev_ptr(grad_out, "float32"),
                                      _dev_ptr(loss_out, "float32"), _stream_handle(stream)))


def mlp_train(theta, feats, labels, steps: int, lr: float, stream=None) -> float:
    """Adam steps on theta in place; returns the final loss."""
    _mlp_inputs(theta, feats, labels)
    loss = C.c_float(0.0)
    check(lib().grng_mlp_train(_dev_ptr(theta, "float32"), _dev_ptr(feats, "float32"), _dev_ptr(labels, "uint8"),
                               feats.shape[0], steps, lr, C.byref(loss), _stream_handle(stream)))
    return float(loss.value)


def mlp_score(theta, feats, stream=None):
    """Scores (bf16 weights, float32 accumulation) as a float32 device tensor."""
    import torch
    _mlp_inputs(theta, feats)
    out = torch.empty(feats.shape[0], dtype=torch.float32, device=feats.device)
    n = feats.shape[0]
    check(lib().grng_mlp_score(_dev_ptr(theta, "float32"), _dev_ptr(feats, "float32") if n else None, n,
                               _dev_ptr(out, "float32") if n else None, _stream_handle(stream)))
    return out


class Index:
    """An exact RNG / GRNG index over device-resident points (see include/grng.h)."""

    def __init__(self, points, grid_exp: int, precision: int = PREC_FP64, witness_order: int = ORDER_DISTANCE,
                 use_graph: int = 0, autotune: int = 0, stage4_pivots: int = 0, vgrng_pivots: int = 0,
                 metric: int = METRIC_L2, graph: int = GRAPH_RNG, beta: float = 0.0, stream=None):
        """beta: the beta of graph=GRAPH_BETA, a multiple of 1/4 in [1, 16] (ignored otherwise)."""
        self._h = C.c_void_p()
        self._stream = stream
        bq = 0
        if graph == GRAPH_BETA:
            bq = int(round(beta * 4))
            if bq != beta * 4:
                raise ValueError("beta must be a multiple of 1/4")
        opt = Options(grid_exp=grid_exp, precision=precision, witness_order=witness_order, use_graph=use_graph,
                      autotune=autotune, stage4_pivots=stage4_pivots, vgrng_pivots=vgrng_pivots, metric=metric,
                      graph=graph, beta_quarters=bq)
        n, d = points.shape
        check(lib().grng_create(C.byref(self._h), _dev_ptr(points, "float32", 2), n, d,
                                _stream_handle(stream), C.byref(opt)))
        self.d = d

    def build_grng_layer(self, layer: int, pivot_ids, radii) -> None:
        m = pivot_ids.numel()
        if radii.numel() != m:
            raise ValueError("pivot_ids and radii differ in length")
        check(lib().grng_build_grng_layer(self._h, layer, _dev_ptr(pivot_ids, "int32", 1),
                                          _dev_ptr(radii, "float32", 1), m))

    def build_rng(self) -> None:
        check(lib().grng_build_rng(self._h))

    def insert_batch(self, points) -> None:
        check(lib().grng_insert_batch(self._h, _dev_ptr(points, "float32", 2), points.shape[0]))

    def insert_pivots(self, layer: int, pivot_ids, radii) -> None:
        """Add pivots (ascending point ids, not yet pivots of `layer`) with their radii to a built layer."""
        m = pivot_ids.numel()
        if radii.numel() != m:
            raise ValueError("pivot_ids and radii differ in length")
        check(lib().grng_insert_pivots(self._h, layer, _dev_ptr(pivot_ids, "int32", 1),
                                       _dev_ptr(radii, "float32", 1), m))

    def orphans(self):
        """Ids of the points without a parent in the finest layer (int32 device tensor, ascending)."""
        import torch
        n = C.c_int64(0)
        st = lib().grng_get_orphans(self._h, None, 0, C.byref(n))
        if st not in (GRNG_OK, GRNG_ECAPACITY):
            check(st)
        out = torch.empty(max(n.value, 1), dtype=torch.int32, device="cuda")
        n2 = C.c_int64(0)
        check(lib().grng_get_orphans(self._h, _dev_ptr(out, "int32") if n.value else None, n.value, C.byref(n2)))
        return out[:n.value]

    def query_neighbors(self, queries):
        """Returns (offsets int64 [nq+1], neighbours int32 [total]) as device tensors."""
        import torch
        nq = queries.shape[0]
        dev = queries.device
        offsets = torch.empty(nq + 1, dtype=torch.int64, device=dev)
        cap = max(16 * nq, 1)
        for _ in range(2):
            nbrs = torch.empty(cap, dtype=torch.int32, device=dev)
            needed = C.c_int64(0)
            st = lib().grng_query_neighbors(self._h, _dev_ptr(queries, "float32", 2), nq, _dev_ptr(offsets, "int64"),
                                            _dev_ptr(nbrs, "int32"), cap, C.byref(needed))
            if st == -5:
                cap = int(needed.value)
                continue
            check(st)
            return offsets, nbrs[:int(needed.value)]
        raise GrngError(-5, "query output kept growing")

    def num_edges(self, layer: int = -1) -> int:
        ne = C.c_int64(0)
        st = lib().grng_get_edges(self._h, layer, None, 0, C.byref(ne))
        if st not in (GRNG_OK, -5):
            check(st)
        return int(ne.value)

    def edges(self, layer: int = -1):
        """Canonical edge list as a device int32 tensor [E, 2] (u < v, sorted)."""
        import torch
        ne = self.num_edges(layer)
        out = torch.empty((max(ne, 0), 2), dtype=torch.int32, device="cuda")
        n2 = C.c_int64(0)
        check(lib().grng_get_edges(self._h, layer, _dev_ptr(out, "int32") if ne else None, ne, C.byref(n2)))
        return out

    def log_witness_cells(self, max_pairs: int):
        """Training samples (feats float32 [n, MLP_FEATURES], labels uint8 [n]) from the last build."""
        import torch
        cnt = C.c_int64(0)
        st = lib().grng_log_witness_cells(self._h, max_pairs, None, None, 0, C.byref(cnt))
        if st not in (GRNG_OK, -5):
            check(st)
        n = int(cnt.value)
        feats = torch.empty((n, MLP_FEATURES), dtype=torch.float32, device="cuda")
        labels = torch.empty(n, dtype=torch.uint8, device="cuda")
        if n:
            check(lib().grng_log_witness_cells(self._h, max_pairs, _dev_ptr(feats, "float32"),
                                               _dev_ptr(labels, "uint8"), n, C.byref(cnt)))
        return feats, labels

    def set_scorer(self, theta) -> None:
        if theta.numel() != mlp_params():
            raise ValueError("theta must hold %d parameters" % mlp_params())
        check(lib().grng_set_scorer(self._h, _dev_ptr(theta, "float32")))

    def stats(self) -> dict:
        st = Stats()
        check(lib().grng_get_stats(self._h, C.byref(st)))
        return st.as_dict()

    def close(self) -> None:
        if self._h:
            lib().grng_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
