"""Layout quality on the GPU (sections 2.5-2.6): k-means labels and pass
counts bit-exact against the oracle, AQ exact, NMI within 1e-12."""
import numpy as np
import pytest

import oracle
from paper_2310_11186_amd import tsgne

pytestmark = pytest.mark.gpu


def blobs(n, k, seed, spread):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-50, 50, (k, 2))
    lab = rng.integers(0, k, n)
    return (centres[lab] + spread * rng.standard_normal((n, 2))).astype(np.float32), lab.astype(np.int32)


KM_CASES = [(300, 3, 1.0, 300), (5000, 12, 4.0, 300), (20000, 200, 2.0, 300), (20000, 30, 8.0, 5),
            (257, 1, 1.0, 10), (1000, 1024, 1.0, 50)]


@pytest.mark.parametrize("n,k,spread,max_iter", KM_CASES)
def test_kmeans_bit_exact(gpu, n, k, spread, max_iter):
    import torch
    Y, _ = blobs(n, min(k, 40), n + k, spread)
    seeds = np.random.default_rng(k).choice(n, k, replace=k > n).astype(np.int32)
    labels, iters = tsgne.tsgne_kmeans(torch.from_numpy(Y).to(gpu), torch.from_numpy(seeds).to(gpu), max_iter)
    ol, oit = oracle.kmeans(Y, seeds, max_iter)
    assert iters == oit
    assert np.array_equal(labels.cpu().numpy(), ol)


def test_kmeans_degenerate(gpu):
    import torch
    Y = np.ones((100, 2), np.float32)                       # one point, flat box
    seeds = np.array([0, 5, 7], np.int32)
    labels, iters = tsgne.tsgne_kmeans(torch.from_numpy(Y).to(gpu), torch.from_numpy(seeds).to(gpu))
    ol, oit = oracle.kmeans(Y, seeds)
    assert iters == oit == 2 and np.array_equal(labels.cpu().numpy(), ol)
    line = np.stack([np.linspace(0, 1, 64), np.zeros(64)], 1).astype(np.float32)   # flat y axis
    seeds = np.array([0, 63, 31, 31], np.int32)                                    # a repeated seed
    labels, iters = tsgne.tsgne_kmeans(torch.from_numpy(line).to(gpu), torch.from_numpy(seeds).to(gpu))
    ol, oit = oracle.kmeans(line, seeds)
    assert iters == oit and np.array_equal(labels.cpu().numpy(), ol)


def test_kmeans_full_size(gpu):
    import torch
    Y, _ = blobs(300_000, 50, 3, 3.0)
    seeds = np.random.default_rng(9).choice(300_000, 50, replace=False).astype(np.int32)
    labels, iters = tsgne.tsgne_kmeans(torch.from_numpy(Y).to(gpu), torch.from_numpy(seeds).to(gpu), 100)
    ol, oit = oracle.kmeans(Y, seeds, 100)
    assert iters == oit and np.array_equal(labels.cpu().numpy(), ol)


@pytest.mark.parametrize("n,ka,kb,seed", [(1000, 4, 4, 0), (50000, 40, 37, 1), (20000, 200, 200, 2),
                                          (3000, 1, 1, 3), (10, 3, 5000, 4)])
def test_nmi_matches_oracle(gpu, n, ka, kb, seed):
    import torch
    rng = np.random.default_rng(seed)
    a = rng.integers(0, ka, n).astype(np.int32)
    b = np.where(rng.random(n) < 0.7, a % kb, rng.integers(0, kb, n)).astype(np.int32)
    got = tsgne.tsgne_nmi(torch.from_numpy(a).to(gpu), ka, torch.from_numpy(b).to(gpu), kb)
    assert abs(got - oracle.nmi(a, ka, b, kb)) <= 1e-12


@pytest.mark.parametrize("n,labels,grid,p,spread", [(2000, 5, 10, 0.6, 3.0), (100000, 40, 20, 0.5, 5.0),
                                                    (100000, 200, 64, 0.8, 1.0), (50, 3, 1, 0.3, 1.0),
                                                    (5000, 2, 4096, 0.5, 1.0)])
def test_aq_matches_oracle(gpu, n, labels, grid, p, spread):
    import torch
    Y, lab = blobs(n, labels, n + grid, spread)
    got = tsgne.tsgne_aq(torch.from_numpy(Y).to(gpu), torch.from_numpy(lab).to(gpu), labels, grid, p)
    assert got == oracle.aq(Y, lab, labels, grid, p)


def test_aq_flat_axis_and_edges(gpu):
    import torch
    line = np.array([[0, 0], [1, 0], [2, 0], [3, 0]], np.float32)
    lab = np.array([0, 1, 0, 1], np.int32)
    got = tsgne.tsgne_aq(torch.from_numpy(line).to(gpu), torch.from_numpy(lab).to(gpu), 2, 3, 0.5)
    assert got == oracle.aq(line, lab, 2, 3, 0.5) == pytest.approx(2 / 9)


def test_quality_rejects(gpu):
    import torch
    Y = torch.zeros((10, 2), dtype=torch.float32, device=gpu)
    lab = torch.zeros(10, dtype=torch.int32, device=gpu)
    with pytest.raises(tsgne.TsgneError) as e:
        tsgne.tsgne_kmeans(Y, torch.tensor([10], dtype=torch.int32, device=gpu))
    assert e.value.status == tsgne.TSGNE_E_INVAL
    with pytest.raises(tsgne.TsgneError) as e:
        tsgne.tsgne_kmeans(Y, torch.zeros(1025, dtype=torch.int32, device=gpu))
    assert e.value.status == tsgne.TSGNE_E_INVAL
    Yn = Y.clone()
    Yn[3, 1] = float("nan")
    with pytest.raises(tsgne.TsgneError) as e:
        tsgne.tsgne_kmeans(Yn, torch.tensor([0], dtype=torch.int32, device=gpu))
    assert e.value.status == tsgne.TSGNE_E_NONFINITE
    with pytest.raises(tsgne.TsgneError) as e:
        tsgne.tsgne_aq(Yn, lab, 1, 4, 0.5)
    assert e.value.status == tsgne.TSGNE_E_NONFINITE
    bad = lab.clone()
    bad[2] = 3
    with pytest.raises(tsgne.TsgneError) as e:
        tsgne.tsgne_aq(Y, bad, 3, 4, 0.5)
    assert e.value.status == tsgne.TSGNE_E_INVAL
    with pytest.raises(tsgne.TsgneError) as e:
        tsgne.tsgne_nmi(lab, 1, bad, 3)
    assert e.value.status == tsgne.TSGNE_E_INVAL
