"""Seeded synthetic inputs for the t-SGNE loop: graphs, embeddings, initial layouts.

This module holds no arithmetic of the method itself; it only draws inputs.
Both the HIP path and the FP64 oracle receive the same arrays from it.

The paper measures on LFR graphs and Network Repository / SNAP datasets
(experiments, Tables 1-3) that are not available here.  Stochastic block models
stand in for them: a plain SBM (equal communities) for the small case, and a
degree-corrected SBM with power-law degree propensities, log-normal community
sizes and LFR's mixing parameter mu = 0.18 (the value the paper uses for its
LFR graphs) for the large ones.  Node ids are randomly permuted after
generation, so memory locality is not given for free.

Embeddings follow the t-SGNE premise (section 2.2): nodes close in the graph
should be close in R^d, so each node's vector is its community centre
(N(0, 4 I)) plus isotropic Gaussian noise.  Initial layouts are N(0, 1e-4 I).

Every draw uses numpy's Philox counter-based generator keyed by an explicit
seed, so any run is reproducible from (config, seed).
"""
from __future__ import annotations

import dataclasses
import math
import re

import numpy as np

MASTER_SEED = 2310_11186


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=np.uint64(seed), counter=np.array([0, 0, 0, stream], np.uint64)))


@dataclasses.dataclass
class GraphInput:
    """An undirected graph as an edge list plus its node embedding and Y0."""
    n: int
    edges: np.ndarray        # int32[m, 2], u != v, each unordered pair once
    labels: np.ndarray       # int32[n] ground-truth community of each node
    X: np.ndarray            # float32[n, d] row-major
    Y0: np.ndarray           # float32[n, 2]
    name: str = ""

    @property
    def d(self) -> int:
        return int(self.X.shape[1])


def _permute(n: int, edges: np.ndarray, labels: np.ndarray, rng: np.random.Generator):
    perm = rng.permutation(n).astype(np.int64)        # old id -> new id
    e = perm[edges.astype(np.int64)]
    lab = np.empty_like(labels)
    lab[perm] = labels
    return e.astype(np.int32), lab


def _unique_pairs_first(keys: np.ndarray, want: int) -> np.ndarray:
    """The first `want` distinct keys in order of first appearance."""
    _, first = np.unique(keys, return_index=True)
    first.sort()
    return keys[first[:want]]


def sbm(sizes, p_in: float, p_out: float, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Plain SBM: each unordered pair is an edge with probability p_in inside a
    community and p_out across.  Returns (edges int32[m,2], labels int32[n])."""
    rng = _rng(seed, 1)
    sizes = np.asarray(sizes, np.int64)
    n = int(sizes.sum())
    labels = np.repeat(np.arange(len(sizes), dtype=np.int32), sizes)
    iu, ju = np.triu_indices(n, k=1)
    same = labels[iu] == labels[ju]
    prob = np.where(same, p_in, p_out)
    keep = rng.random(iu.shape[0]) < prob
    edges = np.stack([iu[keep], ju[keep]], axis=1).astype(np.int32)
    return _permute(n, edges, labels, _rng(seed, 2))


def sbm_sparse(n: int, n_comm: int, avg_deg: float, mu: float, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """SBM with equal communities and a target average degree, sampled edge by
    edge (for graphs too large for the all-pairs draw).  A fraction 1-mu of
    edges is intra-community.  Exactly round(n*avg_deg/2) distinct edges."""
    rng = _rng(seed, 3)
    sizes = np.full(n_comm, n // n_comm, np.int64)
    sizes[: n % n_comm] += 1
    labels = np.repeat(np.arange(n_comm, dtype=np.int32), sizes)
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    m = int(round(n * avg_deg / 2))
    keys = np.zeros(0, np.int64)
    while True:
        k = max(2 * (m - keys.shape[0]), 1024)
        intra = rng.random(k) >= mu
        c = rng.integers(0, n_comm, size=k)
        u_in = starts[c] + (rng.random(k) * sizes[c]).astype(np.int64)
        v_in = starts[c] + (rng.random(k) * sizes[c]).astype(np.int64)
        u_out = rng.integers(0, n, size=k)
        v_out = rng.integers(0, n, size=k)
        u = np.where(intra, u_in, u_out)
        v = np.where(intra, v_in, v_out)
        ok = (u != v) & (intra | (labels[u] != labels[v]))
        a, b = np.minimum(u[ok], v[ok]), np.maximum(u[ok], v[ok])
        keys = _unique_pairs_first(np.concatenate([keys, a * n + b]), m)
        if keys.shape[0] >= m:
            break
    edges = np.stack([keys // n, keys % n], axis=1).astype(np.int32)
    return _permute(n, edges, labels, _rng(seed, 4))


def lognormal_sizes(n: int, n_comm: int, rng: np.random.Generator, min_size: int = 2) -> np.ndarray:
    """Community sizes proportional to exp(N(0,1)), largest-remainder rounding
    to sum n, each at least min_size."""
    w = np.exp(rng.standard_normal(n_comm))
    spare = n - min_size * n_comm
    raw = w / w.sum() * spare
    base = np.floor(raw).astype(np.int64)
    rem = spare - int(base.sum())
    order = np.argsort(-(raw - base), kind="stable")
    base[order[:rem]] += 1
    return base + min_size


def dcsbm(n: int, m: int, gamma: float, n_comm: int, mu: float, seed: int,
          theta_min: float = 2.0) -> tuple[np.ndarray, np.ndarray]:
    """Degree-corrected SBM with exactly m distinct undirected edges.

    theta_i: discrete power law with exponent gamma, theta >= theta_min,
    truncated at n^(1/(gamma-1)).  An edge is intra-community with probability
    1-mu (community chosen in proportion to its total theta, endpoints in
    proportion to theta inside it), otherwise inter-community (endpoints in
    proportion to theta over all nodes, same-community draws rejected).
    Self-loops and repeats are dropped and sampling continues until m
    distinct edges exist; the first m in draw order are kept."""
    rng = _rng(seed, 5)
    sizes = lognormal_sizes(n, n_comm, rng)
    labels = np.repeat(np.arange(n_comm, dtype=np.int32), sizes)
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    tmax = n ** (1.0 / (gamma - 1.0))
    theta = np.floor(theta_min * rng.random(n) ** (-1.0 / (gamma - 1.0)))
    theta = np.minimum(theta, math.floor(tmax)).astype(np.float64)
    cum_all = np.cumsum(theta)
    comm_w = np.add.reduceat(theta, starts)
    cum_comm = np.cumsum(comm_w)
    keys = np.zeros(0, np.int64)
    while True:
        k = max(int(1.3 * (m - keys.shape[0])), 4096)
        intra = rng.random(k) >= mu
        c = np.searchsorted(cum_comm, rng.random(k) * cum_comm[-1], side="right")
        c = np.minimum(c, n_comm - 1)
        lo = np.where(c > 0, cum_all[starts[c] - 1], 0.0)
        hi = cum_all[starts[c] + sizes[c] - 1]
        u_in = np.searchsorted(cum_all, lo + rng.random(k) * (hi - lo), side="right")
        v_in = np.searchsorted(cum_all, lo + rng.random(k) * (hi - lo), side="right")
        u_out = np.searchsorted(cum_all, rng.random(k) * cum_all[-1], side="right")
        v_out = np.searchsorted(cum_all, rng.random(k) * cum_all[-1], side="right")
        u = np.minimum(np.where(intra, u_in, u_out), n - 1)
        v = np.minimum(np.where(intra, v_in, v_out), n - 1)
        ok = (u != v) & (intra | (labels[u] != labels[v]))
        a, b = np.minimum(u[ok], v[ok]), np.maximum(u[ok], v[ok])
        keys = _unique_pairs_first(np.concatenate([keys, a * n + b]), m)
        if keys.shape[0] >= m:
            break
    edges = np.stack([keys // n, keys % n], axis=1).astype(np.int32)
    return _permute(n, edges, labels, _rng(seed, 6))


def embedding(labels: np.ndarray, d: int, noise_std: float, seed: int, centre_std: float = 2.0) -> np.ndarray:
    """x_i = mu_{c(i)} + noise_std * N(0, I), mu_c ~ N(0, centre_std^2 I); float32[n, d]."""
    rng = _rng(seed, 7)
    n_comm = int(labels.max()) + 1 if labels.size else 0
    centres = centre_std * rng.standard_normal((n_comm, d))
    X = centres[labels] + noise_std * rng.standard_normal((labels.shape[0], d))
    return np.ascontiguousarray(X, dtype=np.float32)


def initial_layout(n: int, seed: int, std: float = 0.01) -> np.ndarray:
    """Y0 ~ N(0, std^2 I) in 2-D (std 0.01 = variance 1e-4); float32[n, 2]."""
    rng = _rng(seed, 8)
    return np.ascontiguousarray(std * rng.standard_normal((n, 2)), dtype=np.float32)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    description: str
    n_iter: int
    exaggeration_iters: int
    perplexity: float = 30.0
    early_exaggeration: float = 12.0


WORKLOADS = {
    "sbm2k": Workload("sbm2k", "SBM 2,000 nodes, 4 x 500, p_in 0.02, p_out 0.0005, d=16", 500, 125),
    "dcsbm20k": Workload("dcsbm20k", "DC-SBM 20,000 nodes, 80,000 edges, gamma 2.5, 20 communities, d=64",
                         1000, 250),
    "dcsbm100k": Workload("dcsbm100k", "DC-SBM 100,000 nodes, 400,000 edges, gamma 2.5, 50 communities, d=128",
                          1000, 250),
    "dcsbm300k": Workload("dcsbm300k", "DC-SBM 300,000 nodes, 1,000,000 edges, gamma 2.3, 200 communities, d=128",
                          1000, 250),
    # scale points beyond the paper-scale graph, sized like its largest
    # inputs (about 1.1M nodes / 3M edges and 3M nodes / 4.9M edges)
    "dcsbm1m": Workload("dcsbm1m", "DC-SBM 1,000,000 nodes, 3,000,000 edges, gamma 2.3, 500 communities, d=128",
                        1000, 250),
    "dcsbm3m": Workload("dcsbm3m", "DC-SBM 3,000,000 nodes, 5,000,000 edges, gamma 2.3, 1000 communities, d=64",
                        1000, 250),
}


def make(name: str, seed: int | None = None) -> GraphInput:
    """Build a named workload.  Default seeds: master seed + workload index."""
    if name == "sbm2k":
        s = MASTER_SEED + 1 if seed is None else seed
        edges, labels = sbm([500] * 4, 0.02, 0.0005, s)
        X = embedding(labels, 16, 1.0, s)
        return GraphInput(2000, edges, labels, X, initial_layout(2000, s), name)
    if name == "dcsbm20k":
        s = MASTER_SEED + 23 if seed is None else seed
        edges, labels = dcsbm(20_000, 80_000, 2.5, 20, 0.18, s)
        X = embedding(labels, 64, 0.5, s)
        return GraphInput(20_000, edges, labels, X, initial_layout(20_000, s), name)
    if name == "dcsbm100k":
        s = MASTER_SEED + 2 if seed is None else seed
        edges, labels = dcsbm(100_000, 400_000, 2.5, 50, 0.18, s)
        X = embedding(labels, 128, 0.5, s)
        return GraphInput(100_000, edges, labels, X, initial_layout(100_000, s), name)
    if name == "dcsbm300k":
        s = MASTER_SEED + 3 if seed is None else seed
        edges, labels = dcsbm(300_000, 1_000_000, 2.3, 200, 0.18, s)
        X = embedding(labels, 128, 0.5, s)
        return GraphInput(300_000, edges, labels, X, initial_layout(300_000, s), name)
    if name == "dcsbm1m":
        s = MASTER_SEED + 21 if seed is None else seed
        edges, labels = dcsbm(1_000_000, 3_000_000, 2.3, 500, 0.18, s)
        X = embedding(labels, 128, 0.5, s)
        return GraphInput(1_000_000, edges, labels, X, initial_layout(1_000_000, s), name)
    if name == "dcsbm3m":
        s = MASTER_SEED + 22 if seed is None else seed
        edges, labels = dcsbm(3_000_000, 5_000_000, 2.3, 1000, 0.18, s)
        X = embedding(labels, 64, 0.5, s)
        return GraphInput(3_000_000, edges, labels, X, initial_layout(3_000_000, s), name)
    m = re.fullmatch(r"dcsbm_n(\d+)", name)
    if m:
        # a DC-SBM of any size: average degree 8, gamma 2.5, about 1,000 nodes per community, d = 32
        n = int(m.group(1))
        s = MASTER_SEED + 24 if seed is None else seed
        edges, labels = dcsbm(n, 4 * n, 2.5, max(2, n // 1000), 0.18, s)
        X = embedding(labels, 32, 0.5, s)
        return GraphInput(n, edges, labels, X, initial_layout(n, s), name)
    raise KeyError(name)


def batch_workload(count: int = 256, seed: int | None = None, n_min: int = 500, n_max: int = 50_000,
                   d: int = 64) -> list[GraphInput]:
    """Many independent SBM graphs: node counts log-uniform in [n_min, n_max],
    average degree uniform in [3, 8], 4-40 equal communities each, mixing 0.18,
    d-dim embeddings (community centre + N(0, 0.25 I))."""
    s = MASTER_SEED + 4 if seed is None else seed
    rng = _rng(s, 9)
    out = []
    for k in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        avg = float(rng.uniform(3.0, 8.0))
        comm = int(rng.integers(4, 41))
        edges, labels = sbm_sparse(n, min(comm, n // 2), avg, 0.18, s * 1000 + k)
        X = embedding(labels, d, 0.5, s * 1000 + k)
        out.append(GraphInput(n, edges, labels, X, initial_layout(n, s * 1000 + k), "batch%d" % k))
    return out


def serving_request_specs(count: int, seed: int | None = None, n_min: int = 1_000,
                          n_max: int = 200_000) -> list[tuple]:
    """The drawn parameters of each request of a serving stream, in order:
    (index, n, average degree, communities, d, SBM or DC-SBM, seed base)."""
    s = MASTER_SEED + 5 if seed is None else seed
    rng = _rng(s, 10)
    out = []
    for k in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        avg = float(rng.uniform(2.0, 8.0))
        comm = int(rng.integers(4, 41))
        d = 64 if rng.random() < 0.5 else 128
        plain = bool(rng.random() < 0.5)
        out.append((k, n, avg, comm, d, plain, s))
    return out


def serving_request(spec: tuple) -> GraphInput:
    """One request of a serving stream from its drawn parameters."""
    k, n, avg, comm, d, plain, s = spec
    if plain:
        edges, labels = sbm_sparse(n, comm, avg, 0.18, s * 1000 + k)
    else:
        edges, labels = dcsbm(n, int(round(n * avg / 2)), 2.5, comm, 0.18, s * 1000 + k)
    X = embedding(labels, d, 0.5, s * 1000 + k)
    return GraphInput(n, edges, labels, X, initial_layout(n, s * 1000 + k), "req%d" % k)


def serving_requests(count: int, seed: int | None = None, n_min: int = 1_000, n_max: int = 200_000) -> list[GraphInput]:
    """Layout requests: node counts log-uniform in [n_min, n_max], average degree
    uniform in [2, 8], half plain SBM (4-40 equal communities, mixing 0.18) and
    half DC-SBM (power law 2.5, 4-40 log-normal communities), embeddings of 64
    or 128 dimensions (half each)."""
    return [serving_request(spec) for spec in serving_request_specs(count, seed, n_min, n_max)]


def small_sbm(n: int, n_comm: int, avg_deg: float, d: int, seed: int, mu: float = 0.18) -> GraphInput:
    """A small seeded SBM test case with a given size and average degree."""
    edges, labels = sbm_sparse(n, n_comm, avg_deg, mu, seed)
    X = embedding(labels, d, 1.0, seed)
    return GraphInput(n, edges, labels, X, initial_layout(n, seed), "sbm%d" % n)


def small_dcsbm(n: int, m: int, gamma: float, n_comm: int, d: int, seed: int) -> GraphInput:
    edges, labels = dcsbm(n, m, gamma, n_comm, 0.18, seed)
    X = embedding(labels, d, 0.5, seed)
    return GraphInput(n, edges, labels, X, initial_layout(n, seed), "dcsbm%d" % n)


def snowball_sample(gi: GraphInput, size: int, seed: int) -> GraphInput:
    """The subgraph induced by the nodes a BFS from seeded random roots reaches
    first (until `size` nodes): a sample that keeps the graph's local density.
    Nodes keep their relative order; X, labels and Y0 are the sampled rows."""
    from collections import deque
    rng = np.random.default_rng(seed)
    n = gi.n
    size = min(size, n)
    adj = [[] for _ in range(n)]
    for u, v in gi.edges:
        adj[u].append(v)
        adj[v].append(u)
    seen = np.zeros(n, bool)
    order = []
    while len(order) < size:
        root = int(rng.integers(0, n))
        if seen[root]:
            continue
        seen[root] = True
        q = deque([root])
        while q and len(order) < size:
            u = q.popleft()
            order.append(u)
            for v in adj[u]:
                if not seen[v]:
                    seen[v] = True
                    q.append(v)
    nodes = np.array(sorted(order[:size]), np.int64)
    remap = -np.ones(n, np.int64)
    remap[nodes] = np.arange(size)
    e = remap[gi.edges.astype(np.int64)]
    e = e[(e[:, 0] >= 0) & (e[:, 1] >= 0)].astype(np.int32)
    return GraphInput(size, e, gi.labels[nodes], np.ascontiguousarray(gi.X[nodes]), np.ascontiguousarray(gi.Y0[nodes]),
                      "%s_snowball%d" % (gi.name, size))
