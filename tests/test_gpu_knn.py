"""G_knn,G (section 2.2, eq. (7)) on the GPU: bit-exact against the oracle's
per-node BFS, then the affinities built on it."""
import numpy as np
import pytest

import oracle
from paper_2310_11186_amd import synth, tsgne

pytestmark = pytest.mark.gpu


def device_csr(gi, gpu):
    import torch
    rp, col = tsgne.tsgne_csr_from_edges(gi.n, gi.edges)
    return rp, col, torch.from_numpy(rp).to(gpu), torch.from_numpy(col).to(gpu)


@pytest.mark.parametrize("kind,n,k", [("sbm", 500, 1), ("sbm", 500, 5), ("sbm", 1200, 30), ("dcsbm", 3000, 90),
                                      ("dcsbm", 3000, 256), ("sbm", 300, 256)])
def test_knn_graph_bit_exact(gpu, kind, n, k):
    if kind == "sbm":
        gi = synth.small_sbm(n, 4, 3.0, 4, 13)
    else:
        gi = synth.small_dcsbm(n, 3 * n, 2.3, 10, 4, 13)     # hubs and isolated nodes
    rp, col, d_rp, d_col = device_csr(gi, gpu)
    krp, kcol = tsgne.tsgne_knn_graph(d_rp, d_col, k)
    orp, ocol = oracle.knn_graph(rp, col, k)
    assert np.array_equal(krp.cpu().numpy(), orp)
    assert np.array_equal(kcol.cpu().numpy(), ocol)


def test_knn_graph_full_size(gpu):
    """The benchmark's construction: the 300,000-node, 1,000,000-edge graph
    with k = 90 (46M entries), bit-exact against the oracle."""
    gi = synth.make("dcsbm300k")
    rp, col, d_rp, d_col = device_csr(gi, gpu)
    krp, kcol = tsgne.tsgne_knn_graph(d_rp, d_col, 90)
    orp, ocol = oracle.knn_graph(rp, col, 90)
    assert np.array_equal(krp.cpu().numpy(), orp)
    assert np.array_equal(kcol.cpu().numpy(), ocol)


def test_affinities_on_knn_graph(gpu):
    gi = synth.small_dcsbm(2500, 7500, 2.4, 12, 8, 21)
    rp, col, d_rp, d_col = device_csr(gi, gpu)
    krp, kcol = tsgne.tsgne_knn_graph(d_rp, d_col, 45)
    import torch
    g = tsgne.tsgne_build_P(krp, kcol, torch.from_numpy(gi.X).to(gpu), 15.0)
    orp, ocol = oracle.knn_graph(rp, col, 45)
    oP, _ = oracle.build_P(orp, ocol, gi.X, 15.0)
    P = g.export()["P"]
    assert np.linalg.norm(P - oP) <= 1e-6 * np.linalg.norm(oP)
    Y = np.random.default_rng(2).standard_normal((gi.n, 2)).astype(np.float32)
    grad, _ = tsgne.tsgne_gradient(g, torch.from_numpy(Y).to(gpu), 1.0)
    og, _ = oracle.gradient(orp, ocol, oP, Y.astype(np.float64), 1.0)
    assert np.linalg.norm(grad.cpu().numpy() - og) <= 1e-5 * np.linalg.norm(og)


def test_knn_graph_rejects(gpu):
    import torch
    gi = synth.small_sbm(100, 2, 3.0, 4, 1)
    rp, col, d_rp, d_col = device_csr(gi, gpu)
    with pytest.raises(tsgne.TsgneError):
        tsgne.tsgne_knn_graph(d_rp, d_col, 0)
    with pytest.raises(tsgne.TsgneError):
        tsgne.tsgne_knn_graph(d_rp, d_col, 257)
    bad = col.copy()
    bad[0], bad[1] = bad[1], bad[0]                  # unsorted row
    with pytest.raises(tsgne.TsgneError) as e:
        tsgne.tsgne_knn_graph(d_rp, torch.from_numpy(bad).to(gpu), 5)
    assert e.value.status == tsgne.TSGNE_E_GRAPH
