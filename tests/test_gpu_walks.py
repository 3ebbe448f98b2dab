"""Random-walk P (section 2.1) on the GPU: the walks' support and P
bit-exact against the oracle (same Philox4x32-10 stream on both sides), and
the t-SGNE gradient on it within the usual bar."""
import numpy as np
import pytest

import oracle
from bars import GRAD_TOL, Z_TOL
from paper_2310_11186_amd import synth, tsgne

pytestmark = pytest.mark.gpu


def path_edges(n):
    return np.stack([np.arange(n - 1), np.arange(1, n)], 1).astype(np.int32)


def both(gpu, n, edges, X, walks, length, seed):
    import torch
    rp, col = tsgne.tsgne_csr_from_edges(n, edges)
    g = tsgne.tsgne_build_P_walks(torch.from_numpy(rp).to(gpu), torch.from_numpy(col).to(gpu),
                                  torch.from_numpy(X).to(gpu), walks, length, seed)
    ex = g.export()
    orp, ocol, oP = oracle.walk_P(rp, col, X, walks, length, seed)
    return g, ex, (orp, ocol, oP)


CASES = [
    ("sbm500", lambda: synth.small_sbm(500, 4, 3.0, 8, 1), 10, 1, 7),
    ("sbm500", lambda: synth.small_sbm(500, 4, 3.0, 8, 1), 10, 3, 8),
    ("sbm_sparse", lambda: synth.small_sbm(800, 6, 1.5, 4, 2), 16, 6, 9),        # isolated nodes
    ("dcsbm_hubs", lambda: synth.small_dcsbm(3000, 9000, 2.2, 10, 16, 3), 8, 5, 10),
    ("dcsbm_hubs", lambda: synth.small_dcsbm(3000, 9000, 2.2, 10, 16, 3), 64, 2, 2**40 + 3),
]


@pytest.mark.parametrize("name,make,walks,length,seed", CASES,
                         ids=["%s-w%d-l%d" % (c[0], c[2], c[3]) for c in CASES])
def test_walk_P_bit_exact(gpu, name, make, walks, length, seed):
    gi = make()
    g, ex, (orp, ocol, oP) = both(gpu, gi.n, gi.edges, gi.X, walks, length, seed)
    assert np.array_equal(ex["row_ptr"], orp)
    assert np.array_equal(ex["col"], ocol)
    assert np.array_equal(ex["P"], oP)
    assert np.all(ex["beta"] == 0)
    g.close()


def test_walk_P_full_size(gpu):
    """The benchmark's construction: 32 walks of 3 steps from every node of the
    300,000-node, 1,000,000-edge graph, bit-exact against the oracle."""
    gi = synth.make("dcsbm300k")
    g, ex, (orp, ocol, oP) = both(gpu, gi.n, gi.edges, gi.X, 32, 3, synth.MASTER_SEED + 9)
    assert np.array_equal(ex["row_ptr"], orp)
    assert np.array_equal(ex["col"], ocol)
    assert np.array_equal(ex["P"], oP)
    g.close()


def test_walk_P_path_and_no_edges(gpu):
    import torch
    n = 200
    X = np.random.default_rng(0).standard_normal((n, 3)).astype(np.float32)
    g, ex, (orp, ocol, oP) = both(gpu, n, path_edges(n), X, 12, 10, 5)
    assert np.array_equal(ex["row_ptr"], orp) and np.array_equal(ex["col"], ocol) and np.array_equal(ex["P"], oP)
    g.close()
    rp = torch.zeros(n + 1, dtype=torch.int32, device=gpu)
    g = tsgne.tsgne_build_P_walks(rp, torch.zeros(0, dtype=torch.int32, device=gpu), torch.from_numpy(X).to(gpu),
                                  4, 3, 1)
    assert g.info() == (n, 0)                       # every walk stays put: no support
    g.close()


def test_walk_P_larger_and_gradient(gpu):
    import torch
    gi = synth.small_dcsbm(20000, 80000, 2.5, 30, 32, 4)
    g, ex, (orp, ocol, oP) = both(gpu, gi.n, gi.edges, gi.X, 16, 3, 77)
    assert np.array_equal(ex["row_ptr"], orp) and np.array_equal(ex["col"], ocol) and np.array_equal(ex["P"], oP)
    Y = np.random.default_rng(3).standard_normal((gi.n, 2)).astype(np.float32)
    grad, Z = tsgne.tsgne_gradient(g, torch.from_numpy(Y).to(gpu), 1.0)
    og, oZ = oracle.gradient(orp, ocol, oP.astype(np.float64), Y.astype(np.float64), 1.0)
    assert np.linalg.norm(grad.cpu().numpy() - og) <= GRAD_TOL * np.linalg.norm(og)
    assert abs(Z.item() / oZ - 1) <= Z_TOL
    g.close()


def test_walk_P_rejects(gpu):
    import torch
    gi = synth.small_sbm(100, 2, 3.0, 4, 1)
    rp, col = tsgne.tsgne_csr_from_edges(gi.n, gi.edges)
    d_rp, d_col, d_X = (torch.from_numpy(a).to(gpu) for a in (rp, col, gi.X))
    for walks, length in ((0, 3), (3, 0), (3, 5000)):
        with pytest.raises(tsgne.TsgneError) as e:
            tsgne.tsgne_build_P_walks(d_rp, d_col, d_X, walks, length, 1)
        assert e.value.status == tsgne.TSGNE_E_INVAL
    bad = col.copy()
    bad[0], bad[1] = bad[1], bad[0]
    with pytest.raises(tsgne.TsgneError) as e:
        tsgne.tsgne_build_P_walks(d_rp, torch.from_numpy(bad).to(gpu), d_X, 3, 3, 1)
    assert e.value.status == tsgne.TSGNE_E_GRAPH
