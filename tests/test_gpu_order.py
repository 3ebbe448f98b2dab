"""Locality renumbering on the GPU: the Morton order bit-exact against the
oracle, the renumbered CSR bit-exact against the oracle's CSR builder on the
relabelled edges, row permutations exact, and the t-SGNE gradient equivariant
under the renumbering."""
import numpy as np
import pytest

import oracle
from paper_2310_11186_amd import synth, tsgne

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,d,seed", [(1, 3, 0), (1000, 1, 1), (1000, 2, 2), (5000, 3, 3), (100000, 8, 4),
                                      (20000, 16, 5), (3000, 128, 6)])
def test_locality_order_bit_exact(gpu, n, d, seed):
    import torch
    X = np.random.default_rng(seed).standard_normal((n, d)).astype(np.float32)
    if n > 10:
        X[5] = X[7]                      # a tie
        X[:, 0][X[:, 0] > 2.0] = 2.0     # many ties on one axis
    perm = tsgne.tsgne_locality_order(torch.from_numpy(X).to(gpu))
    assert np.array_equal(perm.cpu().numpy(), oracle.locality_order(X))


def relabelled_csr(gi, perm):
    inv = np.empty(gi.n, np.int64)
    inv[perm] = np.arange(gi.n)
    return oracle.csr_from_edges(gi.n, inv[gi.edges.astype(np.int64)].astype(np.int32))


@pytest.mark.parametrize("which", ["locality", "random"])
def test_permute_graph_bit_exact(gpu, which):
    import torch
    gi = synth.small_dcsbm(20000, 70000, 2.3, 20, 8, 11)
    rp, col = tsgne.tsgne_csr_from_edges(gi.n, gi.edges)
    if which == "locality":
        perm = tsgne.tsgne_locality_order(torch.from_numpy(gi.X).to(gpu))
    else:
        perm = torch.from_numpy(np.random.default_rng(1).permutation(gi.n).astype(np.int32)).to(gpu)
    nrp, ncol = tsgne.tsgne_permute_graph(torch.from_numpy(rp).to(gpu), torch.from_numpy(col).to(gpu), perm)
    orp, ocol = relabelled_csr(gi, perm.cpu().numpy())
    assert np.array_equal(nrp.cpu().numpy(), orp) and np.array_equal(ncol.cpu().numpy(), ocol)


def test_permute_rows_and_equivariance(gpu):
    import torch
    gi = synth.small_sbm(6000, 12, 6.0, 16, 12)
    rp, col = tsgne.tsgne_csr_from_edges(gi.n, gi.edges)
    d_rp, d_col, d_X = (torch.from_numpy(a).to(gpu) for a in (rp, col, gi.X))
    perm = tsgne.tsgne_locality_order(d_X)
    p = perm.cpu().numpy()
    Xp = tsgne.tsgne_permute_rows(d_X, perm)
    assert np.array_equal(Xp.cpu().numpy(), gi.X[p])
    Y = np.random.default_rng(4).standard_normal((gi.n, 2)).astype(np.float32)
    Yp = tsgne.tsgne_permute_rows(torch.from_numpy(Y).to(gpu), perm)
    assert np.array_equal(tsgne.tsgne_permute_rows(Yp, perm, inverse=True).cpu().numpy(), Y)
    nrp, ncol = tsgne.tsgne_permute_graph(d_rp, d_col, perm)
    g0 = tsgne.tsgne_build_P(d_rp, d_col, d_X, 30.0)
    g1 = tsgne.tsgne_build_P(nrp, ncol, Xp, 30.0)
    grad0, Z0 = tsgne.tsgne_gradient(g0, torch.from_numpy(Y).to(gpu), 12.0)
    grad1, Z1 = tsgne.tsgne_gradient(g1, Yp, 12.0)
    back = tsgne.tsgne_permute_rows(grad1, perm, inverse=True).cpu().numpy()
    g = grad0.cpu().numpy()
    assert np.linalg.norm(back - g) <= 1e-6 * np.linalg.norm(g)
    assert abs(Z1.item() / Z0.item() - 1) <= 1e-9
    g0.close()
    g1.close()


def test_order_rejects(gpu):
    import torch
    gi = synth.small_sbm(100, 2, 3.0, 4, 1)
    rp, col = tsgne.tsgne_csr_from_edges(gi.n, gi.edges)
    d_rp, d_col = torch.from_numpy(rp).to(gpu), torch.from_numpy(col).to(gpu)
    bad = torch.arange(gi.n, dtype=torch.int32, device=gpu)
    bad[3] = 4                                          # 4 twice, 3 missing
    with pytest.raises(tsgne.TsgneError) as e:
        tsgne.tsgne_permute_graph(d_rp, d_col, bad)
    assert e.value.status == tsgne.TSGNE_E_INVAL
    X = torch.zeros((10, 2), dtype=torch.float32, device=gpu)
    X[2, 1] = float("inf")
    with pytest.raises(tsgne.TsgneError) as e:
        tsgne.tsgne_locality_order(X)
    assert e.value.status == tsgne.TSGNE_E_NONFINITE
