"""CPU-side checks of the C-ABI library: it loads, exports every symbol the
header declares, and its host-only paths (CSR helper, parameter defaults,
argument validation that fails before any device work) behave as documented.
No compute call reaches the device here."""
import os
import re

import numpy as np
import pytest

import oracle
from paper_2310_11186_amd import tsgne

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    with open(os.path.join(ROOT, "include", "tsgne.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"TSGNE_API\s+[\w\s\*]*?\b(tsgne_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = tsgne.lib()
    declared = header_symbols()
    assert len(declared) >= 12
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(tsgne.EXPORTED) == declared


def test_only_declared_symbols_are_exported():
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", tsgne.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = sorted({ln.split()[-1] for ln in out.splitlines() if " T " in ln and "tsgne" in ln})
    assert exported == header_symbols()


def test_params_default():
    p = tsgne.tsgne_params_default()
    assert p.early_exaggeration == 12.0 and p.exaggeration_iters == 250
    assert p.momentum_early == 0.5 and p.momentum_late == pytest.approx(0.8)
    assert p.min_gain == pytest.approx(0.01) and p.learning_rate == 0.0
    assert p.precision == tsgne.TSGNE_PREC_SPLIT and p.kl_every == 0
    assert p.repulsion == tsgne.TSGNE_REPULSION_AUTO and p.tile_rows == 0


@pytest.mark.parametrize("seed", range(4))
def test_host_csr_helper_matches_oracle_builder(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 200))
    m = int(rng.integers(0, 600))
    uv = rng.integers(0, n, size=(m, 2)).astype(np.int32)   # repeats and self-loops included
    a_rp, a_col = tsgne.tsgne_csr_from_edges(n, uv)
    b_rp, b_col = oracle.csr_from_edges(n, uv)
    assert np.array_equal(a_rp, b_rp)
    assert np.array_equal(a_col, b_col)


def test_host_csr_helper_rejects_bad_input():
    with pytest.raises(tsgne.TsgneError) as e:
        tsgne.tsgne_csr_from_edges(3, np.array([[0, 3]]))
    assert e.value.status == tsgne.TSGNE_E_INVAL
    with pytest.raises(tsgne.TsgneError):
        tsgne.tsgne_csr_from_edges(-1, np.zeros((0, 2)))


def test_argument_validation_before_device_work():
    import ctypes
    L = tsgne.lib()
    out = ctypes.c_void_p(None)
    dummy = ctypes.c_void_p(16)
    # n < 1, d < 1, perplexity <= 1, null pointers: rejected on the host
    assert L.tsgne_build_P(0, 0, dummy, dummy, dummy, 4, 30.0, None, ctypes.byref(out)) == tsgne.TSGNE_E_INVAL
    assert L.tsgne_build_P(5, 4, dummy, dummy, dummy, 0, 30.0, None, ctypes.byref(out)) == tsgne.TSGNE_E_INVAL
    assert L.tsgne_build_P(5, 4, dummy, dummy, dummy, 4, 1.0, None, ctypes.byref(out)) == tsgne.TSGNE_E_INVAL
    assert L.tsgne_build_P(5, 4, None, dummy, dummy, 4, 30.0, None, ctypes.byref(out)) == tsgne.TSGNE_E_INVAL
    assert L.tsgne_build_P(5, -1, dummy, dummy, dummy, 4, 30.0, None, ctypes.byref(out)) == tsgne.TSGNE_E_INVAL
    assert b"perplexity" in L.tsgne_last_error() or True
    p = tsgne.tsgne_params_default()
    assert L.tsgne_step(None, dummy, dummy, dummy, 0, ctypes.byref(p), None, None, None) == tsgne.TSGNE_E_INVAL
    assert L.tsgne_run(None, dummy, 10, ctypes.byref(p), None, None) == tsgne.TSGNE_E_INVAL
    k = ctypes.c_double(0)
    assert L.tsgne_kl(None, dummy, ctypes.byref(k), None) == tsgne.TSGNE_E_INVAL
    assert L.tsgne_kl_noalloc(None, dummy, dummy, None) == tsgne.TSGNE_E_INVAL
    # batches with a tile per graph: null arrays, an empty batch, no steps to time
    one = (ctypes.c_void_p * 1)(None)
    it = (ctypes.c_int32 * 1)(10)
    assert L.tsgne_batch_run_tiles(None, one, it, it, 1, ctypes.byref(p), None) == tsgne.TSGNE_E_INVAL
    assert L.tsgne_batch_run_tiles(one, one, it, it, 0, ctypes.byref(p), None) == tsgne.TSGNE_E_INVAL
    assert L.tsgne_batch_run_tiles(one, one, it, it, 1, ctypes.byref(p), None) == tsgne.TSGNE_E_INVAL   # null graph
    ms = ctypes.c_double(0)
    assert L.tsgne_autotune_tiles(one, one, 1, ctypes.byref(p), 3, None, None, ctypes.byref(ms), ctypes.byref(ms),
                                  None) == tsgne.TSGNE_E_INVAL                                       # no output
    assert L.tsgne_autotune_tiles(one, one, 1, ctypes.byref(p), 0, None, it, None, None, None) == tsgne.TSGNE_E_INVAL
    buf = ctypes.create_string_buffer(16)
    assert L.tsgne_server_error(None, 1, buf, 16) == tsgne.TSGNE_E_INVAL
    lv = ctypes.c_int32(7)
    sp = L.tsgne_shortest_path_embedding
    assert sp(5, 4, dummy, dummy, 0, dummy, 2.0, dummy, ctypes.byref(lv), None) == tsgne.TSGNE_E_INVAL   # d < 1
    assert lv.value == 0
    assert sp(5, 4, dummy, dummy, 257, dummy, 2.0, dummy, None, None) == tsgne.TSGNE_E_INVAL             # d > 256
    assert sp(5, 4, dummy, dummy, 3, dummy, float("nan"), dummy, None, None) == tsgne.TSGNE_E_INVAL      # NaN l0
    assert sp(5, 4, dummy, dummy, 3, None, 2.0, dummy, None, None) == tsgne.TSGNE_E_INVAL                # targets
    assert sp(0, 0, dummy, dummy, 3, dummy, 2.0, dummy, None, None) == tsgne.TSGNE_E_INVAL               # n < 1
    assert L.tsgne_graph_free(None) == tsgne.TSGNE_OK
    # given-P graphs: sizes, the row_ptr span and P's values are checked on the host
    rp = np.array([0, 1, 2], np.int32)
    col = np.array([1, 0], np.int32)
    good = np.array([0.5, 0.5], np.float32)
    fhp = L.tsgne_graph_from_host_P
    assert fhp(0, 0, rp.ctypes.data, col.ctypes.data, good.ctypes.data, None, ctypes.byref(out)) == tsgne.TSGNE_E_INVAL
    assert fhp(2, -1, rp.ctypes.data, col.ctypes.data, good.ctypes.data, None, ctypes.byref(out)) == tsgne.TSGNE_E_INVAL
    assert fhp(2, 2, rp.ctypes.data, col.ctypes.data, None, None, ctypes.byref(out)) == tsgne.TSGNE_E_INVAL
    assert fhp(2, 2, rp.ctypes.data, col.ctypes.data, good.ctypes.data, None, None) == tsgne.TSGNE_E_INVAL
    assert fhp(2, 3, rp.ctypes.data, col.ctypes.data, good.ctypes.data, None, ctypes.byref(out)) == tsgne.TSGNE_E_GRAPH
    for bad in ([-0.5, 0.5], [float("nan"), 0.5], [float("inf"), 0.5]):
        b = np.array(bad, np.float32)
        assert fhp(2, 2, rp.ctypes.data, col.ctypes.data, b.ctypes.data, None, ctypes.byref(out)) == tsgne.TSGNE_E_INVAL
    assert out.value is None
    sh = ctypes.c_void_p(None)
    for args in [(0, 0, 1, 0), (10, 1, 1, 0), (10, -1, 2, 0), (10, 0, 0, 0), (10, 0, 1, 5), (10, 0, 70000, 0)]:
        assert L.tsgne_shard_create(*args, ctypes.byref(sh)) == tsgne.TSGNE_E_INVAL
        assert sh.value is None
    assert L.tsgne_shard_create(10, 0, 1, 0, None) == tsgne.TSGNE_E_INVAL
    assert L.tsgne_shard_repulsion(None, dummy, 0, dummy, dummy, None) == tsgne.TSGNE_E_INVAL
    assert L.tsgne_shard_info(None, None, None, None) == tsgne.TSGNE_E_INVAL
    assert L.tsgne_shard_set_timing(None, 1) == tsgne.TSGNE_E_INVAL
    assert L.tsgne_shard_timing(None, None, None) == tsgne.TSGNE_E_INVAL
    assert L.tsgne_shard_free(None) == tsgne.TSGNE_OK
    assert L.tsgne_status_string(tsgne.TSGNE_E_GRAPH) == b"TSGNE_E_GRAPH"


def test_repulsion_plan_on_the_host():
    # the automatic tile follows the measured crossovers: 1 row per lane up to
    # 3,500 nodes, 2 up to 11,000, then the tiles-per-SIMD cost model
    # (15 rows at the 300K benchmark graph, 1M and 3M; 12 at 150K, 16 at 400K)
    for n, R in [(1, 1), (2000, 1), (3500, 1), (3501, 2), (11000, 2), (20000, 4), (100000, 8),
                 (150000, 12), (300000, 15), (400000, 16), (1000000, 15), (3000000, 15)]:
        r, tiles, nbytes = tsgne.tsgne_repulsion_plan(n)
        assert r == R, (n, r)
        nb = -(-n // (64 * r))
        assert tiles == nb * (nb + 1) // 2
        assert nbytes == 8 * nb * nb * 64 * r
    # a fixed tile and the direct kernel (the whole square of tiles)
    r, tiles, nbytes = tsgne.tsgne_repulsion_plan(5000, 8, tsgne.TSGNE_REPULSION_DIRECT)
    assert (r, tiles, nbytes) == (8, 100, 8 * 10 * 10 * 512)
    # partial buffers as the design states them: about 0.75 GB at 300K, 75 GB at 3M
    assert abs(tsgne.tsgne_repulsion_plan(300000)[2] / 1e9 - 0.75) < 0.02
    assert abs(tsgne.tsgne_repulsion_plan(3000000)[2] / 1e9 - 75.0) < 0.5
    for bad in [(0, 0), (100, 3), (100, 32)]:
        with pytest.raises(tsgne.TsgneError) as e:
            tsgne.tsgne_repulsion_plan(*bad)
        assert e.value.status == tsgne.TSGNE_E_INVAL


def test_traffic_is_reported_only_for_the_counted_kernel():
    """bench.py attaches the committed HBM counter figure only to a run of the
    kernel instantiation it was counted on (same source, tile size, precision
    and variant), and that instantiation is the one the default 300K
    benchmark launches."""
    import json
    import os

    import bench
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "profiles",
                        "repulsion_dcsbm300k_traffic.json")
    with open(path) as f:
        rec = json.load(f)
    R = tsgne.tsgne_repulsion_plan(300_000, 0, tsgne.TSGNE_REPULSION_AUTO)[0]
    assert rec["kernel"] == bench.repulse_kernel_name(R)
    assert bench.measured_traffic("dcsbm300k", bench.repulse_kernel_name(R + 1)) is None
    assert bench.measured_traffic("dcsbm300k", bench.repulse_kernel_name(R, split=False)) is None
    assert bench.measured_traffic("dcsbm300k", bench.repulse_kernel_name(R, symmetric=False)) is None
    if rec["kernel_source_hash"] == bench.kernel_source_hash():
        assert bench.measured_traffic("dcsbm300k", rec["kernel"]) == rec["bytes_per_launch"]
    else:
        assert bench.measured_traffic("dcsbm300k", rec["kernel"]) is None


def test_serving_summaries():
    """The serving statistics bench.py reports: nearest-rank percentiles (the
    server's own definition), size deciles and the slowest requests."""
    import bench
    assert bench.nearest_rank([5, 1, 3, 2, 4], 0.5) == 3
    assert bench.nearest_rank(list(range(1, 201)), 0.99) == 198        # 200 values: the third largest
    assert bench.nearest_rank(list(range(1, 49)), 0.99) == 48          # 48 values: the largest
    assert bench.nearest_rank([], 0.5) is None
    sizes = list(range(100, 0, -5))                                    # 20 requests, largest first
    st = {"per_request": [(float(s), 0.5 * s) for s in sizes]}          # latency grows with size
    dec = bench.by_size_decile(sizes, st)
    assert [d["requests"] for d in dec] == [2] * 10
    assert dec[0]["nodes"] == [5, 10] and dec[-1]["nodes"] == [95, 100]
    assert dec[-1]["latency_max_ms"] == 100.0
    slow = bench.slowest(st, sizes, [0.1 * k for k in range(20)], top=3)
    assert [x["request"] for x in slow] == [0, 1, 2]
    assert slow[0]["nodes"] == 100 and slow[0]["queued_ms"] == 50.0 and slow[1]["arrival_s"] == 0.1
