"""Thin ctypes binding of ``libtsgne.so`` (C-ABI in ``include/tsgne.h``).

Argument marshalling only: torch tensors supply device memory (their
``data_ptr()``) and streams (``torch.cuda.Stream.cuda_stream``); every step of
the computation runs in the HIP library.  The library must have been built
(``python -m paper_2310_11186_amd.build``); loading fails loudly otherwise.
Function names follow the C-ABI.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtsgne.so")

TSGNE_OK = 0
TSGNE_E_INVAL = -1
TSGNE_E_GRAPH = -2
TSGNE_E_NOMEM = -3
TSGNE_E_DEVICE = -4
TSGNE_E_NONFINITE = -5
TSGNE_E_BUSY = -6
TSGNE_E_CANCELLED = -7

TSGNE_PREC_SPLIT = 0
TSGNE_PREC_FP32 = 1

TSGNE_REPULSION_AUTO = 0
TSGNE_REPULSION_DIRECT = 1
TSGNE_REPULSION_SYMMETRIC = 2

AUTOTUNE_TILES = (4, 8, 12, 16)   # the autotuner's candidates, in its output order

TSGNE_SHARE_EQUAL = 0
TSGNE_SHARE_SMALLEST_FIRST = 1
TSGNE_SHARE_SHORT_FIRST = 2

# every symbol include/tsgne.h declares
EXPORTED = (
    "tsgne_params_default", "tsgne_repulsion_plan", "tsgne_last_error", "tsgne_status_string", "tsgne_csr_from_edges", "tsgne_knn_graph",
    "tsgne_shortest_path_embedding", "tsgne_kmeans", "tsgne_nmi", "tsgne_aq", "tsgne_build_P",
    "tsgne_build_P_walks", "tsgne_locality_order", "tsgne_permute_graph", "tsgne_permute_rows",
    "tsgne_graph_from_host_P", "tsgne_graph_free", "tsgne_graph_info", "tsgne_graph_export", "tsgne_gradient", "tsgne_step", "tsgne_run",
    "tsgne_kl", "tsgne_kl_noalloc", "tsgne_attraction", "tsgne_batch_run", "tsgne_autotune",
    "tsgne_batch_run_tiles", "tsgne_autotune_tiles", "tsgne_graph_set_timing", "tsgne_graph_timing",
    "tsgne_server_config_default", "tsgne_server_create", "tsgne_server_submit", "tsgne_server_poll",
    "tsgne_server_wait", "tsgne_server_latency", "tsgne_server_error", "tsgne_server_release", "tsgne_server_cancel", "tsgne_server_get_stats",
    "tsgne_server_destroy", "tsgne_shard_create", "tsgne_shard_info", "tsgne_shard_repulsion", "tsgne_shard_set_timing",
    "tsgne_shard_timing", "tsgne_shard_free",
)

TSGNE_PHASES = ("repulsion", "zsum", "attract", "update", "kl")


class TsgneError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (_status_name(status), message))
        self.status = status


class tsgne_params(ctypes.Structure):
    _fields_ = [
        ("early_exaggeration", ctypes.c_float),
        ("exaggeration_iters", ctypes.c_int32),
        ("learning_rate", ctypes.c_float),
        ("momentum_early", ctypes.c_float),
        ("momentum_late", ctypes.c_float),
        ("min_gain", ctypes.c_float),
        ("precision", ctypes.c_int32),
        ("kl_every", ctypes.c_int32),
        ("repulsion", ctypes.c_int32),
        ("tile_rows", ctypes.c_int32),
    ]


class tsgne_timing(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 5), ("launches", ctypes.c_int64 * 5)]


class tsgne_server_config(ctypes.Structure):
    _fields_ = [
        ("hbm_budget", ctypes.c_int64),
        ("max_active", ctypes.c_int32),
        ("max_queue", ctypes.c_int32),
        ("steps_per_round", ctypes.c_int32),
        ("tile_rows", ctypes.c_int32),
        ("params", tsgne_params),
        ("round_ms", ctypes.c_float),
        ("oldest_share", ctypes.c_float),
        ("rest_policy", ctypes.c_int32),
        ("long_ms", ctypes.c_float),
        ("short_share", ctypes.c_float),
    ]


class tsgne_request(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("m", ctypes.c_int64),
        ("edges_h", ctypes.c_void_p),
        ("d", ctypes.c_int32),
        ("X_h", ctypes.c_void_p),
        ("Y0_h", ctypes.c_void_p),
        ("perplexity", ctypes.c_float),
        ("n_iter", ctypes.c_int32),
    ]


class tsgne_server_stats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
        ("cancelled", ctypes.c_int64), ("queued", ctypes.c_int32), ("active", ctypes.c_int32),
        ("hbm_in_use", ctypes.c_int64), ("hbm_budget", ctypes.c_int64), ("rounds", ctypes.c_int64),
        ("busy_s", ctypes.c_double), ("admit_s", ctypes.c_double), ("plan_s", ctypes.c_double),
        ("latency_p50_ms", ctypes.c_double), ("latency_p99_ms", ctypes.c_double),
        ("latency_mean_ms", ctypes.c_double), ("layouts_per_s", ctypes.c_double),
    ]


_lib = None


def lib():
    """Load libtsgne.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libtsgne.so is not built (%s); run `python -m paper_2310_11186_amd.build`" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        st = ctypes.c_int32
        P = ctypes.POINTER(tsgne_params)
        sig = {
            "tsgne_params_default": (None, [P]),
            "tsgne_repulsion_plan": (st, [i32, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i64),
                                          ctypes.POINTER(i64)]),
            "tsgne_last_error": (ctypes.c_char_p, []),
            "tsgne_status_string": (ctypes.c_char_p, [st]),
            "tsgne_csr_from_edges": (st, [i32, i64, vp, vp, vp, ctypes.POINTER(ctypes.c_int64)]),
            "tsgne_build_P": (st, [i32, i64, vp, vp, vp, i32, ctypes.c_float, vp, ctypes.POINTER(vp)]),
            "tsgne_knn_graph": (st, [i32, i64, vp, vp, i32, vp, vp, i64, ctypes.POINTER(i64), vp]),
            "tsgne_shortest_path_embedding": (st, [i32, i64, vp, vp, i32, vp, ctypes.c_double, vp,
                                                   ctypes.POINTER(i32), vp]),
            "tsgne_kmeans": (st, [i32, vp, i32, vp, i32, vp, ctypes.POINTER(i32), vp]),
            "tsgne_nmi": (st, [i32, vp, i32, vp, i32, ctypes.POINTER(ctypes.c_double), vp]),
            "tsgne_aq": (st, [i32, vp, vp, i32, i32, ctypes.c_double, ctypes.POINTER(ctypes.c_double), vp]),
            "tsgne_build_P_walks": (st, [i32, i64, vp, vp, vp, i32, i32, i32, ctypes.c_uint64, vp,
                                         ctypes.POINTER(vp)]),
            "tsgne_locality_order": (st, [i32, vp, i32, vp, vp]),
            "tsgne_permute_graph": (st, [i32, i64, vp, vp, vp, vp, vp, vp]),
            "tsgne_permute_rows": (st, [i32, i32, vp, vp, i32, vp, vp]),
            "tsgne_graph_from_host_P": (st, [i32, i64, vp, vp, vp, vp, ctypes.POINTER(vp)]),
            "tsgne_graph_free": (st, [vp]),
            "tsgne_graph_info": (st, [vp, ctypes.POINTER(i32), ctypes.POINTER(i64)]),
            "tsgne_graph_export": (st, [vp, vp, vp, vp, vp, vp]),
            "tsgne_gradient": (st, [vp, vp, ctypes.c_float, P, vp, vp, vp]),
            "tsgne_step": (st, [vp, vp, vp, vp, i32, P, vp, vp, vp]),
            "tsgne_run": (st, [vp, vp, i32, P, vp, vp]),
            "tsgne_kl": (st, [vp, vp, ctypes.POINTER(ctypes.c_double), vp]),
            "tsgne_kl_noalloc": (st, [vp, vp, vp, vp]),
            "tsgne_attraction": (st, [vp, vp, i32, vp, vp]),
            "tsgne_batch_run": (st, [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(i32), i32, P, vp]),
            "tsgne_autotune": (st, [ctypes.POINTER(vp), ctypes.POINTER(vp), i32, P, i32, ctypes.POINTER(i32),
                                    ctypes.POINTER(ctypes.c_double), vp]),
            "tsgne_batch_run_tiles": (st, [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(i32),
                                           ctypes.POINTER(i32), i32, P, vp]),
            "tsgne_autotune_tiles": (st, [ctypes.POINTER(vp), ctypes.POINTER(vp), i32, P, i32, ctypes.c_char_p,
                                          ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_double), vp]),
            "tsgne_server_config_default": (None, [ctypes.POINTER(tsgne_server_config)]),
            "tsgne_server_create": (st, [ctypes.POINTER(tsgne_server_config), ctypes.POINTER(vp)]),
            "tsgne_server_submit": (st, [vp, ctypes.POINTER(tsgne_request), ctypes.POINTER(ctypes.c_uint64)]),
            "tsgne_server_poll": (st, [vp, ctypes.c_uint64, vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
            "tsgne_server_wait": (st, [vp, ctypes.c_uint64, vp, ctypes.POINTER(i32)]),
            "tsgne_server_latency": (st, [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double)]),
            "tsgne_server_error": (st, [vp, ctypes.c_uint64, ctypes.c_char_p, i32]),
            "tsgne_server_release": (st, [vp, ctypes.c_uint64]),
            "tsgne_server_cancel": (st, [vp, ctypes.c_uint64]),
            "tsgne_server_get_stats": (st, [vp, ctypes.POINTER(tsgne_server_stats)]),
            "tsgne_server_destroy": (st, [vp]),
            "tsgne_shard_create": (st, [i32, i32, i32, i32, ctypes.POINTER(vp)]),
            "tsgne_shard_info": (st, [vp, ctypes.POINTER(i32), ctypes.POINTER(i64), ctypes.POINTER(i64)]),
            "tsgne_shard_repulsion": (st, [vp, vp, i32, vp, vp, vp]),
            "tsgne_shard_set_timing": (st, [vp, i32]),
            "tsgne_shard_timing": (st, [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]),
            "tsgne_shard_free": (st, [vp]),
            "tsgne_graph_set_timing": (st, [vp, i32]),
            "tsgne_graph_timing": (st, [vp, ctypes.POINTER(tsgne_timing)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _status_name(s: int) -> str:
    try:
        return lib().tsgne_status_string(s).decode()
    except Exception:
        return "status %d" % s


def _check(status: int) -> None:
    if status != TSGNE_OK:
        raise TsgneError(status, lib().tsgne_last_error().decode())


def _ptr(t) -> int | None:
    if t is None:
        return None
    return t.data_ptr()


def _stream(stream) -> int | None:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _require(t, dtype, shape=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_cuda:
        raise TypeError("%s must be a device tensor" % name)
    if not t.is_contiguous():
        raise TypeError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))


def tsgne_params_default(**overrides) -> tsgne_params:
    p = tsgne_params()
    lib().tsgne_params_default(ctypes.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def tsgne_repulsion_plan(n: int, tile_rows: int = 0, repulsion: int = TSGNE_REPULSION_AUTO) -> tuple[int, int, int]:
    """(rows per lane, tiles per step, bytes of repulsion partials) for a graph of n nodes (host only)."""
    R, tiles, nbytes = ctypes.c_int32(0), ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib().tsgne_repulsion_plan(int(n), int(tile_rows), int(repulsion), ctypes.byref(R), ctypes.byref(tiles),
                                      ctypes.byref(nbytes)))
    return R.value, tiles.value, nbytes.value


def tsgne_csr_from_edges(n: int, edges) -> tuple[np.ndarray, np.ndarray]:
    """Canonical symmetric CSR (host numpy) of an undirected edge list."""
    uv = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
    m = uv.shape[0]
    row_ptr = np.zeros(n + 1, np.int32)
    col = np.zeros(max(2 * m, 1), np.int32)
    nnz = ctypes.c_int64(0)
    _check(lib().tsgne_csr_from_edges(n, m, uv.ctypes.data, row_ptr.ctypes.data, col.ctypes.data,
                                      ctypes.byref(nnz)))
    return row_ptr, col[: nnz.value].copy()


def tsgne_knn_graph(row_ptr, col, k: int, stream=None):
    """Device CSR (row_ptr, col) of G_knn,G for a device CSR of G (int32 tensors)."""
    import torch
    _require(row_ptr, torch.int32, name="row_ptr")
    _require(col, torch.int32, name="col")
    n = row_ptr.shape[0] - 1
    out_rp = torch.empty(n + 1, dtype=torch.int32, device=row_ptr.device)
    cap = 2 * n * int(k)
    out_col = torch.empty(max(cap, 1), dtype=torch.int32, device=row_ptr.device)
    nnz = ctypes.c_int64(0)
    _check(lib().tsgne_knn_graph(n, col.shape[0], _ptr(row_ptr), _ptr(col) if col.numel() else None, int(k),
                                 _ptr(out_rp), _ptr(out_col), cap, ctypes.byref(nnz), _stream(stream)))
    return out_rp, out_col[: nnz.value].clone()


def tsgne_shortest_path_embedding(row_ptr, col, targets, l0: float = -1.0, stream=None):
    """X float32[n, d] (device) of the ShortestPath embedding (section 2.3, eq. (8)) from a device
    CSR and device int32 targets; l0 < 0 selects sqrt(|E|).  Returns (X, levels launched)."""
    import torch
    _require(row_ptr, torch.int32, name="row_ptr")
    _require(col, torch.int32, name="col")
    _require(targets, torch.int32, name="targets")
    n, d = row_ptr.shape[0] - 1, targets.shape[0]
    X = torch.empty((max(n, 0), d), dtype=torch.float32, device=row_ptr.device)
    levels = ctypes.c_int32(0)
    _check(lib().tsgne_shortest_path_embedding(n, col.shape[0], _ptr(row_ptr), _ptr(col) if col.numel() else None,
                                               d, _ptr(targets), float(l0), _ptr(X), ctypes.byref(levels),
                                               _stream(stream)))
    return X, levels.value


def tsgne_kmeans(Y, seeds, max_iter: int = 300, stream=None):
    """Layout clustering of section 2.5 (Lloyd's k-means from the given seed nodes on
    the quantised layout): returns (labels int32 device tensor, passes made)."""
    import torch
    _require(Y, torch.float32, name="Y")
    _require(seeds, torch.int32, name="seeds")
    n = Y.shape[0]
    labels = torch.empty(max(n, 1), dtype=torch.int32, device=Y.device)
    iters = ctypes.c_int32(0)
    _check(lib().tsgne_kmeans(n, _ptr(Y), seeds.shape[0], _ptr(seeds), int(max_iter), _ptr(labels),
                              ctypes.byref(iters), _stream(stream)))
    return labels[:n], iters.value


def tsgne_nmi(a, ka: int, b, kb: int, stream=None) -> float:
    """NMI of two device labelings (section 2.5, eq. (11))."""
    import torch
    _require(a, torch.int32, name="a")
    _require(b, torch.int32, name="b")
    if a.shape != b.shape:
        raise ValueError("labelings differ in length")
    out = ctypes.c_double(0)
    _check(lib().tsgne_nmi(a.shape[0], _ptr(a), int(ka), _ptr(b), int(kb), ctypes.byref(out), _stream(stream)))
    return out.value


def tsgne_aq(Y, labels, n_labels: int, grid: int, p: float, stream=None) -> float:
    """Aesthetic quality of a device layout (section 2.6, eqs. (12)-(14))."""
    import torch
    _require(Y, torch.float32, name="Y")
    _require(labels, torch.int32, name="labels")
    out = ctypes.c_double(0)
    _check(lib().tsgne_aq(Y.shape[0], _ptr(Y), _ptr(labels), int(n_labels), int(grid), float(p), ctypes.byref(out),
                          _stream(stream)))
    return out.value


def tsgne_locality_order(X, stream=None):
    """perm (int32 device tensor): nodes in Morton order of their leading embedding coordinates."""
    import torch
    _require(X, torch.float32, name="X")
    perm = torch.empty(X.shape[0], dtype=torch.int32, device=X.device)
    _check(lib().tsgne_locality_order(X.shape[0], _ptr(X), X.shape[1], _ptr(perm), _stream(stream)))
    return perm


def tsgne_permute_graph(row_ptr, col, perm, stream=None):
    """(row_ptr, col) of the graph renumbered by perm (new node r = old node perm[r])."""
    import torch
    _require(row_ptr, torch.int32, name="row_ptr")
    _require(col, torch.int32, name="col")
    _require(perm, torch.int32, name="perm")
    n = row_ptr.shape[0] - 1
    out_rp = torch.empty_like(row_ptr)
    out_col = torch.empty(max(col.shape[0], 1), dtype=torch.int32, device=col.device)
    _check(lib().tsgne_permute_graph(n, col.shape[0], _ptr(row_ptr), _ptr(col) if col.numel() else None, _ptr(perm),
                                     _ptr(out_rp), _ptr(out_col), _stream(stream)))
    return out_rp, out_col[: col.shape[0]]


def tsgne_permute_rows(src, perm, inverse: bool = False, stream=None):
    """Row r of the result = src row perm[r] (or, inverse, result row perm[r] = src row r)."""
    import torch
    _require(perm, torch.int32, name="perm")
    if not src.is_cuda or not src.is_contiguous():
        raise TypeError("src must be a contiguous device tensor")
    dst = torch.empty_like(src)
    row_bytes = src[0].numel() * src.element_size() if src.dim() > 1 else src.element_size()
    _check(lib().tsgne_permute_rows(src.shape[0], row_bytes, _ptr(src), _ptr(perm), 1 if inverse else 0, _ptr(dst),
                                    _stream(stream)))
    return dst


class Graph:
    """Owns a tsgne_graph* (freed on close() or garbage collection)."""

    def __init__(self, handle: int):
        self._h = handle

    @property
    def handle(self) -> int:
        if not self._h:
            raise ValueError("graph has been freed")
        return self._h

    def close(self) -> None:
        if self._h:
            lib().tsgne_graph_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> tuple[int, int]:
        n, nnz = ctypes.c_int32(0), ctypes.c_int64(0)
        _check(lib().tsgne_graph_info(self.handle, ctypes.byref(n), ctypes.byref(nnz)))
        return n.value, nnz.value

    def set_timing(self, enable: bool = True) -> None:
        _check(lib().tsgne_graph_set_timing(self.handle, 1 if enable else 0))

    def timing(self) -> dict:
        """{phase: (total ms, launches)} since timing was enabled (synchronising)."""
        t = tsgne_timing()
        _check(lib().tsgne_graph_timing(self.handle, ctypes.byref(t)))
        return {name: (t.ms[k], t.launches[k]) for k, name in enumerate(TSGNE_PHASES)}

    def export(self) -> dict:
        n, nnz = self.info()
        out = {
            "row_ptr": np.zeros(n + 1, np.int32), "col": np.zeros(max(nnz, 1), np.int32),
            "mirror": np.zeros(max(nnz, 1), np.int32), "P": np.zeros(max(nnz, 1), np.float32),
            "beta": np.zeros(n, np.float64),
        }
        _check(lib().tsgne_graph_export(self.handle, out["row_ptr"].ctypes.data, out["col"].ctypes.data,
                                        out["mirror"].ctypes.data, out["P"].ctypes.data, out["beta"].ctypes.data))
        for k in ("col", "mirror", "P"):
            out[k] = out[k][:nnz]
        return out


class Shard:
    """Owns a tsgne_shard*: one GPU's share of a row-sharded repulsion."""

    def __init__(self, n: int, shard: int, n_shards: int, tile_rows: int = 0):
        h = ctypes.c_void_p(None)
        _check(lib().tsgne_shard_create(int(n), int(shard), int(n_shards), int(tile_rows), ctypes.byref(h)))
        self._h = h.value
        self.n = int(n)

    @property
    def handle(self) -> int:
        if not self._h:
            raise ValueError("shard has been freed")
        return self._h

    def close(self) -> None:
        if self._h:
            lib().tsgne_shard_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> tuple[int, int, int]:
        """(tile rows, tiles, ordered pairs) of this shard."""
        R, tiles, pairs = ctypes.c_int32(0), ctypes.c_int64(0), ctypes.c_int64(0)
        _check(lib().tsgne_shard_info(self.handle, ctypes.byref(R), ctypes.byref(tiles), ctypes.byref(pairs)))
        return R.value, tiles.value, pairs.value

    def set_timing(self, enable: bool = True) -> None:
        _check(lib().tsgne_shard_set_timing(self.handle, 1 if enable else 0))

    def timing(self) -> tuple[float, int]:
        """(total ms, launches) of the tile kernel since timing was enabled (synchronising)."""
        ms, k = ctypes.c_double(0.0), ctypes.c_int64(0)
        _check(lib().tsgne_shard_timing(self.handle, ctypes.byref(ms), ctypes.byref(k)))
        return ms.value, k.value

    def repulsion(self, Y, precision: int = TSGNE_PREC_SPLIT, F=None, Z=None, stream=None):
        """(F float64[n, 2], Z float64[1]): this shard's force sums and Z partial at Y (float32[n, 2])."""
        import torch
        _require(Y, torch.float32, (self.n, 2), "Y")
        F = torch.empty((self.n, 2), dtype=torch.float64, device=Y.device) if F is None else F
        Z = torch.empty(1, dtype=torch.float64, device=Y.device) if Z is None else Z
        _require(F, torch.float64, (self.n, 2), "F")
        _require(Z, torch.float64, (1,), "Z")
        _check(lib().tsgne_shard_repulsion(self.handle, _ptr(Y), int(precision), _ptr(F), _ptr(Z), _stream(stream)))
        return F, Z


def tsgne_build_P(row_ptr, col, X, perplexity: float, stream=None) -> Graph:
    """row_ptr int32[n+1], col int32[nnz], X float32[n, d]: device tensors."""
    import torch
    _require(row_ptr, torch.int32, name="row_ptr")
    _require(col, torch.int32, name="col")
    _require(X, torch.float32, name="X")
    n = row_ptr.shape[0] - 1
    if X.dim() != 2 or X.shape[0] != n:
        raise ValueError("X must be [n, d]")
    h = ctypes.c_void_p(None)
    _check(lib().tsgne_build_P(n, col.shape[0], _ptr(row_ptr), _ptr(col) if col.numel() else None, _ptr(X),
                               X.shape[1], float(perplexity), _stream(stream), ctypes.byref(h)))
    return Graph(h.value)


def tsgne_graph_from_host_P(row_ptr, col, P, stream=None) -> Graph:
    """A graph with given joint affinities: row_ptr int32[n+1], col int32[nnz]
    (canonical symmetric CSR) and P float32[nnz] (symmetric), host numpy arrays."""
    row_ptr = np.ascontiguousarray(row_ptr, np.int32)
    col = np.ascontiguousarray(col, np.int32)
    P = np.ascontiguousarray(P, np.float32)
    if P.shape != col.shape:
        raise ValueError("P must be aligned with col")
    h = ctypes.c_void_p(None)
    _check(lib().tsgne_graph_from_host_P(row_ptr.shape[0] - 1, col.shape[0], row_ptr.ctypes.data,
                                         col.ctypes.data if col.size else None, P.ctypes.data if P.size else None,
                                         _stream(stream), ctypes.byref(h)))
    return Graph(h.value)


def tsgne_build_P_walks(row_ptr, col, X, walks: int, length: int, seed: int, stream=None) -> Graph:
    """P from random walks on the device CSR (section 2.1); the graph's CSR is the walks' support."""
    import torch
    _require(row_ptr, torch.int32, name="row_ptr")
    _require(col, torch.int32, name="col")
    _require(X, torch.float32, name="X")
    n = row_ptr.shape[0] - 1
    if X.dim() != 2 or X.shape[0] != n:
        raise ValueError("X must be [n, d]")
    h = ctypes.c_void_p(None)
    _check(lib().tsgne_build_P_walks(n, col.shape[0], _ptr(row_ptr), _ptr(col) if col.numel() else None, _ptr(X),
                                     X.shape[1], int(walks), int(length), ctypes.c_uint64(seed), _stream(stream),
                                     ctypes.byref(h)))
    return Graph(h.value)


def tsgne_gradient(g: Graph, Y, alpha: float = 1.0, params: tsgne_params | None = None, grad=None, Z=None,
                   stream=None):
    """g at Y (float32[n, 2] device) with P scaled by alpha; returns (grad, Z tensor[1] float64)."""
    import torch
    n, _ = g.info()
    _require(Y, torch.float32, (n, 2), "Y")
    grad = torch.empty_like(Y) if grad is None else grad
    Z = torch.empty(1, dtype=torch.float64, device=Y.device) if Z is None else Z
    _require(grad, torch.float32, (n, 2), "grad")
    _require(Z, torch.float64, (1,), "Z")
    _check(lib().tsgne_gradient(g.handle, _ptr(Y), float(alpha), ctypes.byref(params) if params else None,
                                _ptr(grad), _ptr(Z), _stream(stream)))
    return grad, Z


def tsgne_attraction(g: Graph, Y, precision: int = TSGNE_PREC_SPLIT, A=None, stream=None):
    """A_i = sum_j p_ij w_ij (y_i - y_j) at Y (float32[n, 2]); returns float64[n, 2]."""
    import torch
    n, _ = g.info()
    _require(Y, torch.float32, (n, 2), "Y")
    A = torch.empty((n, 2), dtype=torch.float64, device=Y.device) if A is None else A
    _require(A, torch.float64, (n, 2), "A")
    _check(lib().tsgne_attraction(g.handle, _ptr(Y), int(precision), _ptr(A), _stream(stream)))
    return A


def tsgne_step(g: Graph, Y, upd, gains, t: int, params: tsgne_params, grad_out=None, Z_out=None, stream=None):
    import torch
    n, _ = g.info()
    for name, t_ in (("Y", Y), ("upd", upd), ("gains", gains)):
        _require(t_, torch.float32, (n, 2), name)
    if grad_out is not None:
        _require(grad_out, torch.float32, (n, 2), "grad_out")
    if Z_out is not None:
        _require(Z_out, torch.float64, (1,), "Z_out")
    _check(lib().tsgne_step(g.handle, _ptr(Y), _ptr(upd), _ptr(gains), int(t), ctypes.byref(params),
                            _ptr(grad_out), _ptr(Z_out), _stream(stream)))


def tsgne_run(g: Graph, Y, n_iter: int, params: tsgne_params, stream=None) -> np.ndarray:
    """Runs n_iter steps in place on Y; returns the KL trace (empty if kl_every == 0)."""
    import torch
    n, _ = g.info()
    _require(Y, torch.float32, (n, 2), "Y")
    k = n_iter // params.kl_every if params.kl_every > 0 else 0
    trace = np.zeros(max(k, 1), np.float64)
    _check(lib().tsgne_run(g.handle, _ptr(Y), int(n_iter), ctypes.byref(params),
                           trace.ctypes.data if k > 0 else None, _stream(stream)))
    return trace[:k]


def tsgne_kl(g: Graph, Y, stream=None) -> float:
    import torch
    n, _ = g.info()
    _require(Y, torch.float32, (n, 2), "Y")
    out = ctypes.c_double(0.0)
    _check(lib().tsgne_kl(g.handle, _ptr(Y), ctypes.byref(out), _stream(stream)))
    return out.value


def tsgne_kl_noalloc(g: Graph, Y, out, stream=None):
    """KL at Y into out (float64[1] device tensor, caller-owned), in stream
    order, with no allocation and no synchronisation; returns out."""
    import torch
    n, _ = g.info()
    _require(Y, torch.float32, (n, 2), "Y")
    _require(out, torch.float64, (1,), "out")
    _check(lib().tsgne_kl_noalloc(g.handle, _ptr(Y), _ptr(out), _stream(stream)))
    return out


def tsgne_batch_run(graphs, Ys, n_iter, params: tsgne_params, stream=None) -> None:
    """Advances graphs[k] (Graph) on layouts Ys[k] (float32[n_k, 2] device) by
    n_iter[k] steps together (one captured step replayed for the batch)."""
    import torch
    count = len(graphs)
    if len(Ys) != count or len(n_iter) != count:
        raise ValueError("graphs, Ys and n_iter must have the same length")
    for g, Y in zip(graphs, Ys):
        _require(Y, torch.float32, (g.info()[0], 2), "Y")
    hs = (ctypes.c_void_p * count)(*[g.handle for g in graphs])
    ys = (ctypes.c_void_p * count)(*[Y.data_ptr() for Y in Ys])
    it = (ctypes.c_int32 * count)(*[int(k) for k in n_iter])
    _check(lib().tsgne_batch_run(hs, ys, it, count, ctypes.byref(params), _stream(stream)))


def tsgne_autotune(graphs, Ys, params: tsgne_params, steps: int = 3, stream=None) -> tuple[int, list]:
    """(fastest tile_rows, [ms per step for tile_rows 4, 8, 12, 16]) for this batch."""
    count = len(graphs)
    hs = (ctypes.c_void_p * count)(*[g.handle for g in graphs])
    ys = (ctypes.c_void_p * count)(*[Y.data_ptr() for Y in Ys])
    best = ctypes.c_int32(0)
    ms = (ctypes.c_double * len(AUTOTUNE_TILES))()
    _check(lib().tsgne_autotune(hs, ys, count, ctypes.byref(params), int(steps), ctypes.byref(best), ms,
                                _stream(stream)))
    return best.value, list(ms)


def tsgne_batch_run_tiles(graphs, Ys, n_iter, tile_rows, params: tsgne_params, stream=None) -> None:
    """tsgne_batch_run with a tile per graph (tile_rows[k]; 0 = the single-graph plan's choice)."""
    import torch
    count = len(graphs)
    if len(Ys) != count or len(n_iter) != count or len(tile_rows) != count:
        raise ValueError("graphs, Ys, n_iter and tile_rows must have the same length")
    for g, Y in zip(graphs, Ys):
        _require(Y, torch.float32, (g.info()[0], 2), "Y")
    hs = (ctypes.c_void_p * count)(*[g.handle for g in graphs])
    ys = (ctypes.c_void_p * count)(*[Y.data_ptr() for Y in Ys])
    it = (ctypes.c_int32 * count)(*[int(k) for k in n_iter])
    tr = (ctypes.c_int32 * count)(*[int(k) for k in tile_rows])
    _check(lib().tsgne_batch_run_tiles(hs, ys, it, tr, count, ctypes.byref(params), _stream(stream)))


def tsgne_autotune_tiles(graphs, Ys, params: tsgne_params, steps: int = 3, cache_path: str | None = None,
                         stream=None) -> tuple[list, float, float]:
    """(tile rows per graph, ms per step with the best single tile, ms per step tuned): tiles by size
    bucket floor(log2 n), cached by architecture in cache_path (JSON) when given."""
    count = len(graphs)
    hs = (ctypes.c_void_p * count)(*[g.handle for g in graphs])
    ys = (ctypes.c_void_p * count)(*[Y.data_ptr() for Y in Ys])
    out = (ctypes.c_int32 * count)()
    mu, mt = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(lib().tsgne_autotune_tiles(hs, ys, count, ctypes.byref(params), int(steps),
                                      cache_path.encode() if cache_path else None, out, ctypes.byref(mu),
                                      ctypes.byref(mt), _stream(stream)))
    return list(out), mu.value, mt.value


class Server:
    """Continuous-batching layout server (tsgne_server_*).  Requests are host
    numpy arrays; the server copies them in at submission."""

    def __init__(self, hbm_budget: int = 0, max_active: int | None = None, max_queue: int | None = None,
                 steps_per_round: int | None = None, tile_rows: int = 0, params: tsgne_params | None = None,
                 round_ms: float | None = None, oldest_share: float | None = None, rest_policy: int | None = None,
                 long_ms: float | None = None, short_share: float | None = None):
        # arguments left at None keep tsgne_server_config_default's values
        cfg = tsgne_server_config()
        lib().tsgne_server_config_default(ctypes.byref(cfg))
        cfg.hbm_budget = int(hbm_budget)
        if max_active is not None:
            cfg.max_active = int(max_active)
        if max_queue is not None:
            cfg.max_queue = int(max_queue)
        if steps_per_round is not None:
            cfg.steps_per_round = int(steps_per_round)
        cfg.tile_rows = int(tile_rows)
        if round_ms is not None:
            cfg.round_ms = float(round_ms)
        if oldest_share is not None:
            cfg.oldest_share = float(oldest_share)
        if rest_policy is not None:
            cfg.rest_policy = int(rest_policy)
        if long_ms is not None:
            cfg.long_ms = float(long_ms)
        if short_share is not None:
            cfg.short_share = float(short_share)
        if params is not None:
            cfg.params = params
        h = ctypes.c_void_p(None)
        _check(lib().tsgne_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h.value
        self._n = {}

    def submit(self, n: int, edges, X, Y0, perplexity: float = 30.0, n_iter: int = 500) -> int:
        e = np.ascontiguousarray(np.asarray(edges, np.int32).reshape(-1, 2))
        X = np.ascontiguousarray(X, np.float32)
        Y0 = np.ascontiguousarray(Y0, np.float32)
        if X.shape[0] != n or Y0.shape != (n, 2):
            raise ValueError("X must be [n, d] and Y0 [n, 2]")
        rq = tsgne_request(n=n, m=e.shape[0], edges_h=e.ctypes.data if e.size else None, d=X.shape[1],
                           X_h=X.ctypes.data, Y0_h=Y0.ctypes.data, perplexity=float(perplexity),
                           n_iter=int(n_iter))
        t = ctypes.c_uint64(0)
        _check(lib().tsgne_server_submit(self._h, ctypes.byref(rq), ctypes.byref(t)))
        self._n[t.value] = n
        return t.value

    def poll(self, ticket: int):
        """(done, status, Y or None)."""
        Y = np.zeros((self._n[ticket], 2), np.float32)
        done, st = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(lib().tsgne_server_poll(self._h, ticket, Y.ctypes.data, ctypes.byref(done), ctypes.byref(st)))
        if not done.value:
            return False, None, None
        return True, st.value, (Y if st.value == TSGNE_OK else None)

    def wait(self, ticket: int):
        """(status, Y or None), blocking."""
        Y = np.zeros((self._n[ticket], 2), np.float32)
        st = ctypes.c_int32(0)
        _check(lib().tsgne_server_wait(self._h, ticket, Y.ctypes.data, ctypes.byref(st)))
        return st.value, (Y if st.value == TSGNE_OK else None)

    def latency(self, ticket: int) -> tuple[float, float]:
        """(submission to completion, submission to admission) in ms of a finished request."""
        lat, q = ctypes.c_double(0.0), ctypes.c_double(0.0)
        _check(lib().tsgne_server_latency(self._h, ticket, ctypes.byref(lat), ctypes.byref(q)))
        return lat.value, q.value

    def error(self, ticket: int) -> str:
        """The error message of a finished request ('' if it succeeded)."""
        buf = ctypes.create_string_buffer(1024)
        _check(lib().tsgne_server_error(self._h, ticket, buf, len(buf)))
        return buf.value.decode()

    def cancel(self, ticket: int) -> None:
        _check(lib().tsgne_server_cancel(self._h, ticket))

    def release(self, ticket: int) -> None:
        _check(lib().tsgne_server_release(self._h, ticket))
        self._n.pop(ticket, None)

    def stats(self) -> dict:
        st = tsgne_server_stats()
        _check(lib().tsgne_server_get_stats(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in tsgne_server_stats._fields_}

    def close(self) -> None:
        if self._h:
            lib().tsgne_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
