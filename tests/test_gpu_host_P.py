"""Graphs with given affinities (tsgne_graph_from_host_P) through the C-ABI:
the optimisation loop checked on the oracle's own P rounded to FP32, so that
the comparison isolates the loop (gradient, update, KL) from the affinity
construction; round trip and equivalence with a built graph; rejections."""
import numpy as np
import pytest

import oracle
from bars import GRAD_TOL, ROW_TOL, Z_TOL, kl_close, rel_l2, row_error_ratio
from paper_2310_11186_amd import synth, tsgne

pytestmark = pytest.mark.gpu

TRAJ_TOL = 1e-4


def oracle_case(n, seed, perplexity=30.0, kind="dcsbm"):
    if kind == "dcsbm":
        gi = synth.small_dcsbm(n, 3 * n, 2.4, max(2, n // 200), 8, seed)
    else:
        gi = synth.small_sbm(n, 4, 6.0, 8, seed)
    rp, col = oracle.csr_from_edges(gi.n, gi.edges)
    P, _ = oracle.build_P(rp, col, gi.X, perplexity)
    return gi, rp, col, P.astype(np.float32)


@pytest.mark.parametrize("n", [300, 3001])
def test_round_trip_and_structure(gpu, n):
    gi, rp, col, P32 = oracle_case(n, 11)
    g = tsgne.tsgne_graph_from_host_P(rp, col, P32)
    ex = g.export()
    g.close()
    np.testing.assert_array_equal(ex["row_ptr"], rp)
    np.testing.assert_array_equal(ex["col"], col)
    np.testing.assert_array_equal(ex["P"], P32)
    np.testing.assert_array_equal(ex["mirror"], oracle.mirror(rp, col))
    assert not ex["beta"].any()


@pytest.mark.parametrize("n", [300, 3001])
def test_gradient_on_oracle_P(gpu, n):
    import torch
    gi, rp, col, P32 = oracle_case(n, 12)
    g = tsgne.tsgne_graph_from_host_P(rp, col, P32)
    rng = np.random.default_rng(3)
    for Y in (gi.Y0, rng.standard_normal((n, 2)).astype(np.float32),
              (20 * rng.standard_normal((n, 2))).astype(np.float32)):
        for alpha in (1.0, 12.0):
            grad, Z = tsgne.tsgne_gradient(g, torch.from_numpy(Y).to(gpu), alpha)
            og, oZ = oracle.gradient(rp, col, P32.astype(np.float64), Y.astype(np.float64), alpha)
            gg = grad.cpu().numpy()
            assert rel_l2(gg, og) <= GRAD_TOL
            assert row_error_ratio(gg, og, Y, oZ)[0] <= ROW_TOL
            assert abs(Z.item() / oZ - 1.0) <= Z_TOL
    kl = tsgne.tsgne_kl(g, torch.from_numpy(Y).to(gpu))
    assert kl_close(kl, oracle.kl(rp, col, P32.astype(np.float64), Y.astype(np.float64)))
    g.close()


def test_trajectory_on_oracle_P(gpu):
    # 30 steps from Y0 on a 4-community SBM, where the oracle with its state
    # rounded to FP32 after every step stays within 1e-7 of its FP64 run (on
    # the hub-heavy DC-SBM graphs the same drift reaches 5e-2 by step 30:
    # chaos, not rounding), so the FP32 loop must stay within 1e-4
    import torch
    n, steps = 2000, 30
    gi, rp, col, P32 = oracle_case(n, 13, kind="sbm")
    g = tsgne.tsgne_graph_from_host_P(rp, col, P32)
    Y = torch.from_numpy(gi.Y0).to(gpu)
    tsgne.tsgne_run(g, Y, steps, tsgne.tsgne_params_default(exaggeration_iters=125, learning_rate=50.0))
    oY, _, _, _ = oracle.run(rp, col, P32.astype(np.float64), gi.Y0, n_steps=steps, exaggeration_iters=125, eta=50.0)
    g.close()
    assert rel_l2(Y.cpu().numpy(), oY) <= TRAJ_TOL


def test_same_as_a_built_graph(gpu):
    # the loop depends only on the CSR and P: a graph rebuilt from an exported
    # P runs bit for bit like the graph it came from
    import torch
    gi = synth.small_sbm(1500, 4, 6.0, 8, 14)
    rp, col = tsgne.tsgne_csr_from_edges(gi.n, gi.edges)
    built = tsgne.tsgne_build_P(torch.from_numpy(rp).to(gpu), torch.from_numpy(col).to(gpu),
                                torch.from_numpy(gi.X).to(gpu), 30.0)
    given = tsgne.tsgne_graph_from_host_P(rp, col, built.export()["P"])
    p = tsgne.tsgne_params_default(exaggeration_iters=20, learning_rate=40.0)
    Ya = torch.from_numpy(gi.Y0).to(gpu)
    Yb = torch.from_numpy(gi.Y0).to(gpu)
    tsgne.tsgne_run(built, Ya, 60, p)
    tsgne.tsgne_run(given, Yb, 60, p)
    assert torch.equal(Ya, Yb)
    assert tsgne.tsgne_kl(built, Ya) == tsgne.tsgne_kl(given, Yb)
    built.close()
    given.close()


def test_rejects(gpu):
    gi, rp, col, P32 = oracle_case(300, 15)
    bad = P32.copy()
    bad[0] = bad[0] * 0.5 + 1e-6        # one entry changed alone: P no longer symmetric
    with pytest.raises(tsgne.TsgneError) as err:
        tsgne.tsgne_graph_from_host_P(rp, col, bad)
    assert err.value.status == tsgne.TSGNE_E_INVAL
    unsorted = col.copy()
    row = int(np.nonzero(np.diff(rp) >= 2)[0][0])   # a row with two entries or more
    a = int(rp[row])
    unsorted[a], unsorted[a + 1] = unsorted[a + 1], unsorted[a]
    with pytest.raises(tsgne.TsgneError) as err:
        tsgne.tsgne_graph_from_host_P(rp, unsorted, P32)
    assert err.value.status == tsgne.TSGNE_E_GRAPH
    # no edges at all: a valid graph whose nodes feel only repulsion
    g = tsgne.tsgne_graph_from_host_P(np.zeros(11, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
    assert g.info() == (10, 0)
    g.close()
