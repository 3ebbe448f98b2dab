"""ctypes wrapper around the FP64 C oracle (``tsgne_oracle.c``).

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU-baseline timing).  The C
file is compiled with gcc into ``liboracle.so`` beside it when that library is
missing or older than its source.  Every function takes and returns numpy
arrays; floating-point results are float64.

Citations are to Li, Xiao, Zhou, "Efficiently Visualizing Large Graphs"
(arXiv 2310.11186): §2 problem statement, §2.1 eqs. (2)-(5), §2.2 eq. (7).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tsgne_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

__all__ = [
    "build", "lib", "num_threads", "set_threads", "csr_from_edges", "knn_graph", "shortest_path_embedding", "kmeans", "nmi", "aq", "philox4x32_10", "walk_P", "locality_order", "mirror", "edge_sqdist", "calibrate",
    "symmetrise", "build_P", "Z", "gradient", "gradient_rows", "repulsion_terms", "kl", "kl_given_Z", "update", "run", "OracleError",
]


class OracleError(RuntimeError):
    pass


def build(force: bool = False) -> str:
    """Compile the oracle with gcc -O2 (no fast-math), OpenMP over rows."""
    with _lock:
        stale = (not os.path.exists(_LIB)) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)
        if force or stale:
            tmp = _LIB + ".tmp%d" % os.getpid()
            cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-o", tmp, _SRC, "-lm"]
            subprocess.run(cmd, check=True)
            os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        i32, i64, dbl, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
        sig = {
            "oracle_num_threads": (ctypes.c_int, []),
            "oracle_set_threads": (None, [ctypes.c_int]),
            "oracle_csr_from_edges": (ctypes.c_int, [i32, i64, vp, vp, vp, vp]),
            "oracle_mirror": (ctypes.c_int, [i32, i64, vp, vp, vp]),
            "oracle_knn_graph": (ctypes.c_int, [i32, vp, vp, i32, vp, vp, vp]),
            "oracle_shortest_path_embedding": (ctypes.c_int, [i32, vp, vp, i32, vp, dbl, vp]),
            "oracle_kmeans": (ctypes.c_int, [i32, vp, i32, vp, i32, vp, vp]),
            "oracle_philox4x32_10": (None, [vp, vp, vp]),
            "oracle_locality_order": (ctypes.c_int, [i32, vp, i32, vp]),
            "oracle_walk_P": (ctypes.c_int, [i32, vp, vp, vp, i32, i32, i32, ctypes.c_uint64, vp, vp, vp, vp]),
            "oracle_nmi": (dbl, [i32, vp, i32, vp, i32]),
            "oracle_aq": (dbl, [i32, vp, vp, i32, i32, dbl]),
            "oracle_edge_sqdist": (None, [i32, vp, vp, vp, i32, vp]),
            "oracle_calibrate": (None, [i32, vp, vp, dbl, vp, vp]),
            "oracle_symmetrise": (ctypes.c_int, [i32, vp, vp, vp, vp]),
            "oracle_build_P": (ctypes.c_int, [i32, i64, vp, vp, vp, i32, dbl, vp, vp]),
            "oracle_Z": (dbl, [i32, vp]),
            "oracle_gradient": (None, [i32, vp, vp, vp, vp, dbl, vp, vp]),
            "oracle_gradient_rows": (None, [i32, vp, vp, vp, vp, dbl, vp, i32, vp, vp]),
            "oracle_repulsion_terms": (None, [i32, vp, vp, vp, vp, i32, vp, vp]),
            "oracle_kl": (dbl, [i32, vp, vp, vp, vp]),
            "oracle_kl_given_Z": (dbl, [i32, vp, vp, vp, vp, dbl]),
            "oracle_update": (None, [i32, vp, vp, vp, vp, dbl, dbl, dbl]),
            "oracle_run": (None, [i32, vp, vp, vp, vp, vp, vp, i32, i32, dbl, i32, dbl, dbl, dbl, dbl, i32, vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_threads(k: int) -> None:
    lib().oracle_set_threads(int(k))


def csr_from_edges(n: int, edges) -> tuple[np.ndarray, np.ndarray]:
    """Canonical symmetric CSR (row_ptr int32[n+1], col int32[nnz]) of an
    undirected edge list int[m, 2] (§2: G undirected, unweighted)."""
    uv = _i32(np.asarray(edges).reshape(-1, 2))
    m = uv.shape[0]
    row_ptr = np.zeros(n + 1, np.int32)
    col = np.zeros(max(2 * m, 1), np.int32)
    nnz = ctypes.c_int64(0)
    rc = lib().oracle_csr_from_edges(n, m, _p(uv), _p(row_ptr), _p(col), ctypes.byref(nnz))
    if rc != 0:
        raise OracleError("csr_from_edges failed (%d)" % rc)
    return row_ptr, col[: nnz.value].copy()


def knn_graph(row_ptr, col, k: int) -> tuple[np.ndarray, np.ndarray]:
    """Canonical CSR of G_knn,G (§2.2, eq. (7)): i ~ j when either is among the
    other's k smallest nodes by (BFS hop distance, id)."""
    row_ptr, col = _i32(row_ptr), _i32(col)
    n = row_ptr.shape[0] - 1
    out_rp = np.zeros(n + 1, np.int32)
    out_col = np.zeros(max(2 * n * k, 1), np.int32)
    nnz = ctypes.c_int64(0)
    rc = lib().oracle_knn_graph(n, _p(row_ptr), _p(col), int(k), _p(out_rp), _p(out_col), ctypes.byref(nnz))
    if rc != 0:
        raise OracleError("knn_graph failed (%d)" % rc)
    return out_rp, out_col[: nnz.value].copy()


def shortest_path_embedding(row_ptr, col, targets, l0: float) -> np.ndarray:
    """X float32[n, d]: hop distance to each target if <= l0, else l0 + 1 (§2.3, eq. (8))."""
    row_ptr, col, targets = _i32(row_ptr), _i32(col), _i32(targets)
    n, d = row_ptr.shape[0] - 1, targets.shape[0]
    X = np.zeros((n, d), np.float32)
    rc = lib().oracle_shortest_path_embedding(n, _p(row_ptr), _p(col), d, _p(targets), float(l0), _p(X))
    if rc != 0:
        raise OracleError("shortest_path_embedding failed (%d)" % rc)
    return X


def kmeans(Y, seeds, max_iter: int = 300):
    """Labels int32[n] and the number of passes: Lloyd's k-means on the layout
    quantised to its bounding box (section 2.5, readings in the C source)."""
    Y = np.ascontiguousarray(Y, np.float32)
    seeds = _i32(seeds)
    n = Y.shape[0]
    labels = np.zeros(n, np.int32)
    iters = ctypes.c_int32(0)
    rc = lib().oracle_kmeans(n, _p(Y), seeds.shape[0], _p(seeds), int(max_iter), _p(labels), ctypes.byref(iters))
    if rc != 0:
        raise OracleError("kmeans failed (%d)" % rc)
    return labels, iters.value


def nmi(a, ka: int, b, kb: int) -> float:
    """Normalised mutual information of two labelings (section 2.5, eq. (11))."""
    a, b = _i32(a), _i32(b)
    return float(lib().oracle_nmi(a.shape[0], _p(a), int(ka), _p(b), int(kb)))


def aq(Y, labels, n_labels: int, grid: int, p: float) -> float:
    """Aesthetic quality of a layout (section 2.6, eqs. (12)-(14))."""
    Y = np.ascontiguousarray(Y, np.float32)
    labels = _i32(labels)
    return float(lib().oracle_aq(Y.shape[0], _p(Y), _p(labels), int(n_labels), int(grid), float(p)))


def philox4x32_10(ctr, key) -> np.ndarray:
    """One Philox4x32-10 block (Salmon et al. 2011): uint32[4] from a uint32[4] counter and uint32[2] key."""
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().oracle_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def walk_P(row_ptr, col, X, walks: int, length: int, seed: int):
    """(row_ptr, col, P float32) of the random-walk P of section 2.1 (readings in the C source)."""
    row_ptr, col = _i32(row_ptr), _i32(col)
    X = np.ascontiguousarray(X, np.float32)
    n, d = row_ptr.shape[0] - 1, X.shape[1]
    cap = max(2 * n * int(walks), 1)
    orp = np.zeros(n + 1, np.int32)
    ocol = np.zeros(cap, np.int32)
    P = np.zeros(cap, np.float32)
    nnz = ctypes.c_int64(0)
    rc = lib().oracle_walk_P(n, _p(row_ptr), _p(col), _p(X), d, int(walks), int(length), ctypes.c_uint64(seed),
                             _p(orp), _p(ocol), _p(P), ctypes.byref(nnz))
    if rc != 0:
        raise OracleError("walk_P failed (%d)" % rc)
    return orp, ocol[: nnz.value].copy(), P[: nnz.value].copy()


def locality_order(X) -> np.ndarray:
    """perm int32[n]: the nodes in Morton order of their leading embedding coordinates."""
    X = np.ascontiguousarray(X, np.float32)
    n, d = X.shape
    perm = np.zeros(n, np.int32)
    rc = lib().oracle_locality_order(n, _p(X), d, _p(perm))
    if rc != 0:
        raise OracleError("locality_order failed (%d)" % rc)
    return perm


def mirror(row_ptr, col) -> np.ndarray:
    """mirror[e] = position of (j, i) for e = (i, j); raises on a CSR that is
    not canonical or not symmetric."""
    row_ptr, col = _i32(row_ptr), _i32(col)
    n = row_ptr.shape[0] - 1
    out = np.zeros(max(col.shape[0], 1), np.int32)
    rc = lib().oracle_mirror(n, col.shape[0], _p(row_ptr), _p(col), _p(out))
    if rc != 0:
        raise OracleError("graph is not canonical/symmetric (%d)" % rc)
    return out[: col.shape[0]]


def edge_sqdist(row_ptr, col, X) -> np.ndarray:
    row_ptr, col, X = _i32(row_ptr), _i32(col), _f32(X)
    n, d = X.shape
    D = np.zeros(max(col.shape[0], 1), np.float64)
    lib().oracle_edge_sqdist(n, _p(row_ptr), _p(col), _p(X), d, _p(D))
    return D[: col.shape[0]]


def calibrate(row_ptr, D, perplexity: float) -> tuple[np.ndarray, np.ndarray]:
    """(p_{j|i} aligned with col, beta per row) by the perplexity search."""
    row_ptr, D = _i32(row_ptr), _f64(D)
    n = row_ptr.shape[0] - 1
    pc = np.zeros(max(D.shape[0], 1), np.float64)
    beta = np.zeros(n, np.float64)
    lib().oracle_calibrate(n, _p(row_ptr), _p(D), float(perplexity), _p(pc), _p(beta))
    return pc[: D.shape[0]], beta


def symmetrise(row_ptr, col, pcond) -> np.ndarray:
    row_ptr, col, pcond = _i32(row_ptr), _i32(col), _f64(pcond)
    n = row_ptr.shape[0] - 1
    P = np.zeros(max(col.shape[0], 1), np.float64)
    rc = lib().oracle_symmetrise(n, _p(row_ptr), _p(col), _p(pcond), _p(P))
    if rc != 0:
        raise OracleError("symmetrise: graph not symmetric")
    return P[: col.shape[0]]


def build_P(row_ptr, col, X, perplexity: float) -> tuple[np.ndarray, np.ndarray]:
    """(P float64 aligned with col, beta per row): eqs. (2)-(3) over N(i)."""
    row_ptr, col, X = _i32(row_ptr), _i32(col), _f32(X)
    n, d = X.shape
    P = np.zeros(max(col.shape[0], 1), np.float64)
    beta = np.zeros(n, np.float64)
    rc = lib().oracle_build_P(n, col.shape[0], _p(row_ptr), _p(col), _p(X), d, float(perplexity), _p(P), _p(beta))
    if rc != 0:
        raise OracleError("build_P failed (%d)" % rc)
    return P[: col.shape[0]], beta


def Z(Y) -> float:
    Y = _f64(Y)
    return float(lib().oracle_Z(Y.shape[0], _p(Y)))


def gradient(row_ptr, col, P, Y, alpha: float = 1.0) -> tuple[np.ndarray, float]:
    """(g float64[n, 2], Z) at Y; g = 4 sum_j (alpha p_ij - q_ij) w_ij (y_i - y_j)."""
    row_ptr, col, P, Y = _i32(row_ptr), _i32(col), _f64(P), _f64(Y)
    n = Y.shape[0]
    g = np.zeros((n, 2), np.float64)
    z = ctypes.c_double(0.0)
    lib().oracle_gradient(n, _p(row_ptr), _p(col), _p(P), _p(Y), float(alpha), _p(g), ctypes.byref(z))
    return g, z.value


def gradient_rows(row_ptr, col, P, Y, rows, alpha: float = 1.0) -> tuple[np.ndarray, float]:
    """Gradient of the listed rows only (Z still over all pairs)."""
    row_ptr, col, P, Y, rows = _i32(row_ptr), _i32(col), _f64(P), _f64(Y), _i32(rows)
    n = Y.shape[0]
    g = np.zeros((rows.shape[0], 2), np.float64)
    z = ctypes.c_double(0.0)
    lib().oracle_gradient_rows(n, _p(row_ptr), _p(col), _p(P), _p(Y), float(alpha), _p(rows), rows.shape[0],
                               _p(g), ctypes.byref(z))
    return g, z.value


def repulsion_terms(Y, group=None, counted=None, rows=None, with_Z: bool = True):
    """(F float64[rows, 2], Z_part or None): F_i = sum of w_ij^2 (y_i - y_j) and
    Z_part = sum of w_ij over the pairs {i, j} with counted[min(group[i],
    group[j])] (all pairs when group is None); w of eq. (4)."""
    Y = _f64(Y)
    n = Y.shape[0]
    if group is not None:
        group = _i32(group)
        counted = np.ascontiguousarray(counted, dtype=np.uint8)
        if group.shape[0] != n or (n and (group.min() < 0 or group.max() >= counted.shape[0])):
            raise OracleError("group must hold n indices into counted")
    if rows is not None:
        rows = _i32(rows)
        if rows.size and (rows.min() < 0 or rows.max() >= n):
            raise OracleError("row out of range")
    nrows = n if rows is None else rows.shape[0]
    F = np.zeros((max(nrows, 1), 2), np.float64)
    z = ctypes.c_double(0.0)
    lib().oracle_repulsion_terms(n, _p(Y), _p(group) if group is not None else None,
                                 _p(counted) if group is not None else None,
                                 _p(rows) if rows is not None else None, nrows, _p(F),
                                 ctypes.byref(z) if with_Z else None)
    return F[:nrows], (z.value if with_Z else None)


def kl(row_ptr, col, P, Y) -> float:
    row_ptr, col, P, Y = _i32(row_ptr), _i32(col), _f64(P), _f64(Y)
    return float(lib().oracle_kl(Y.shape[0], _p(row_ptr), _p(col), _p(P), _p(Y)))


def kl_given_Z(row_ptr, col, P, Y, Z: float) -> float:
    """KL at Y with Q's normaliser Z supplied (from Z() or gradient*() at the same Y)."""
    row_ptr, col, P, Y = _i32(row_ptr), _i32(col), _f64(P), _f64(Y)
    return float(lib().oracle_kl_given_Z(Y.shape[0], _p(row_ptr), _p(col), _p(P), _p(Y), float(Z)))


def update(Y, U, gains, g, momentum: float, eta: float, min_gain: float = 0.01):
    """One momentum/gains update; returns new (Y, U, gains) as float64 copies."""
    Y, U, gains, g = _f64(Y).copy(), _f64(U).copy(), _f64(gains).copy(), _f64(g)
    lib().oracle_update(Y.shape[0], _p(Y), _p(U), _p(gains), _p(g), float(momentum), float(eta), float(min_gain))
    return Y, U, gains


def run(row_ptr, col, P, Y, U=None, gains=None, t0: int = 0, n_steps: int = 1, early_exaggeration: float = 12.0,
        exaggeration_iters: int = 0, momentum_early: float = 0.5, momentum_late: float = 0.8, eta: float = 50.0,
        min_gain: float = 0.01, kl_every: int = 0):
    """Steps t0 .. t0+n_steps-1; returns (Y, U, gains, kl_trace)."""
    row_ptr, col, P = _i32(row_ptr), _i32(col), _f64(P)
    Y = _f64(Y).copy()
    n = Y.shape[0]
    U = np.zeros_like(Y) if U is None else _f64(U).copy()
    gains = np.ones_like(Y) if gains is None else _f64(gains).copy()
    nk = 0
    if kl_every > 0:
        nk = sum(1 for t in range(t0, t0 + n_steps) if (t + 1) % kl_every == 0)
    trace = np.zeros(max(nk, 1), np.float64)
    lib().oracle_run(n, _p(row_ptr), _p(col), _p(P), _p(Y), _p(U), _p(gains), int(t0), int(n_steps),
                     float(early_exaggeration), int(exaggeration_iters), float(momentum_early), float(momentum_late),
                     float(eta), float(min_gain), int(kl_every), _p(trace) if kl_every > 0 else None)
    return Y, U, gains, trace[:nk]
