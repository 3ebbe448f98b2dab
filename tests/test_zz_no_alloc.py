"""tsgne_kl_noalloc (KL with its scratch in a fixed device array, for callers
that cannot allocate) against tsgne_kl through the C-ABI: two calls in a row,
the second on a smaller graph, each bitwise equal to tsgne_kl at the same
layout (same kernels, same plan) and within the KL bar of the FP64 oracle;
a graph whose plan changed after a step; a graph beyond the array refused."""
import numpy as np
import pytest

import oracle
from bars import kl_close
from paper_2310_11186_amd import synth, tsgne

pytestmark = pytest.mark.gpu


def built(gpu, gi):
    import torch
    rp, col = tsgne.tsgne_csr_from_edges(gi.n, gi.edges)
    g = tsgne.tsgne_build_P(torch.from_numpy(rp).to(gpu), torch.from_numpy(col).to(gpu),
                            torch.from_numpy(gi.X).to(gpu), 30.0)
    return g, rp, col


def test_kl_noalloc_equals_kl(gpu):
    import torch
    big = synth.small_dcsbm(20000, 80000, 2.4, 40, 16, 31)
    small = synth.small_sbm(900, 3, 5.0, 8, 32)
    out = torch.full((1,), float("nan"), dtype=torch.float64, device=gpu)
    for gi, scale in ((big, 3.0), (small, 0.5)):     # the second call on a smaller input
        g, rp, col = built(gpu, gi)
        Y = (scale * np.random.default_rng(gi.n).standard_normal((gi.n, 2))).astype(np.float32)
        dY = torch.from_numpy(Y).to(gpu)
        tsgne.tsgne_kl_noalloc(g, dY, out)           # before the graph's first step: the automatic plan
        torch.cuda.synchronize()
        got = out.item()
        ref = tsgne.tsgne_kl(g, dY)
        assert got == ref, (gi.n, got, ref)
        oP, _ = oracle.build_P(rp, col, gi.X, 30.0)
        assert kl_close(got, oracle.kl(rp, col, oP, Y.astype(np.float64)))
        g.close()


def test_kl_noalloc_follows_the_graphs_plan(gpu):
    import torch
    gi = synth.small_dcsbm(5000, 15000, 2.4, 10, 8, 33)
    g, _, _ = built(gpu, gi)
    p = tsgne.tsgne_params_default(tile_rows=8, exaggeration_iters=5, learning_rate=100.0)
    Y = torch.from_numpy(gi.Y0).to(gpu)
    U, G = torch.zeros_like(Y), torch.ones_like(Y)
    for t in range(10):
        tsgne.tsgne_step(g, Y, U, G, t, p)           # the workspace is now planned with 8 rows per lane
    out = torch.empty(1, dtype=torch.float64, device=gpu)
    s = torch.cuda.Stream(device=gpu)
    s.wait_stream(torch.cuda.current_stream())
    tsgne.tsgne_kl_noalloc(g, Y, out, stream=s)
    s.synchronize()
    assert out.item() == tsgne.tsgne_kl(g, Y)
    g.close()


def test_kl_noalloc_refuses_a_graph_beyond_its_array(gpu):
    import torch
    n = 3_000_000
    g = tsgne.tsgne_graph_from_host_P(np.zeros(n + 1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
    Y = torch.zeros((n, 2), dtype=torch.float32, device=gpu)
    out = torch.empty(1, dtype=torch.float64, device=gpu)
    with pytest.raises(tsgne.TsgneError) as e:
        tsgne.tsgne_kl_noalloc(g, Y, out)
    assert e.value.status == tsgne.TSGNE_E_INVAL and "too large" in str(e.value)
    g.close()
