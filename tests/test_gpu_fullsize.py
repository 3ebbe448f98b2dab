"""Parity at the full sizes of the benchmark workloads, in the launch
configuration bench.py times (default parameters: automatic tile, symmetric
repulsion, precision split).

dcsbm100k (100,000 nodes, 400,000 edges, d = 128): the oracle computes the
whole gradient.  dcsbm300k (300,000 nodes, 1,000,000 edges): the oracle
computes Z over all 9e10 ordered pairs and the gradient of 512 seeded random
rows plus the first and last row and the first row of the last block of every
tile length.  The CSR, mirror index and P are compared in full on both.  Bars
as in tests/bars.py, the per-row gradient bound included.
"""
import numpy as np
import pytest

import oracle
from bars import GRAD_TOL, P_TOL, ROW_TOL, Z_TOL, kl_close, rel_l2, row_error_ratio, sample_rows
from paper_2310_11186_amd import synth, tsgne

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=["dcsbm100k", "dcsbm300k"])
def big(request, gpu):
    import torch
    name = request.param
    gi = synth.make(name)
    rp, col = tsgne.tsgne_csr_from_edges(gi.n, gi.edges)
    g = tsgne.tsgne_build_P(torch.from_numpy(rp).to(gpu), torch.from_numpy(col).to(gpu),
                            torch.from_numpy(gi.X).to(gpu), synth.WORKLOADS[name].perplexity)
    orp, ocol = oracle.csr_from_edges(gi.n, gi.edges)
    oP, obeta = oracle.build_P(orp, ocol, gi.X, synth.WORKLOADS[name].perplexity)
    yield name, gi, g, orp, ocol, oP, obeta
    g.close()


def test_structure_and_P_full(big):
    name, gi, g, orp, ocol, oP, obeta = big
    ex = g.export()
    assert np.array_equal(ex["row_ptr"], orp)
    assert np.array_equal(ex["col"], ocol)
    assert np.array_equal(ex["mirror"], oracle.mirror(orp, ocol))
    assert np.array_equal(ex["P"], ex["P"][ex["mirror"]])
    assert rel_l2(ex["P"], oP) <= P_TOL
    assert abs(float(ex["P"].astype(np.float64).sum()) - 1.0) <= 1e-5
    fin = np.isfinite(obeta) & (obeta > 0)
    np.testing.assert_allclose(ex["beta"][fin], obeta[fin], rtol=1e-11)


@pytest.mark.parametrize("state", ["y0", "spread"])
def test_gradient_Z_KL_full_size(big, gpu, state):
    import torch
    name, gi, g, orp, ocol, oP, _ = big
    if state == "y0":
        Y = gi.Y0
    else:
        Y = (20.0 * np.random.default_rng(3).standard_normal((gi.n, 2))).astype(np.float32)
    p = tsgne.tsgne_params_default()
    dY = torch.from_numpy(Y).to(gpu)
    alpha = 12.0 if state == "y0" else 1.0
    grad, Z = tsgne.tsgne_gradient(g, dY, alpha, p)
    grad = grad.cpu().numpy()
    if gi.n <= 100_000:
        rows = None
        og, oZ = oracle.gradient(orp, ocol, oP, Y.astype(np.float64), alpha)
        gg = grad
    else:
        rows = sample_rows(gi.n, 512, 11)
        assert rows.shape[0] > 512 and rows[-1] == gi.n - 1
        og, oZ = oracle.gradient_rows(orp, ocol, oP, Y.astype(np.float64), rows, alpha)
        gg = grad[rows]
    assert rel_l2(gg, og) <= GRAD_TOL
    worst, row = row_error_ratio(gg, og, Y, oZ, rows)
    assert worst <= ROW_TOL, (row, worst)
    assert abs(Z.item() / oZ - 1.0) <= Z_TOL
    kl = tsgne.tsgne_kl(g, dY)
    okl = oracle.kl_given_Z(orp, ocol, oP, Y.astype(np.float64), oZ)
    assert kl_close(kl, okl), (kl, okl)
