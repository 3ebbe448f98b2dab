"""One GPU's share of a row-sharded repulsion (tsgne_shard_*) through the
C-ABI: every shard's force sums and Z partial against the FP64 oracle over the
same pairs, the shards' tiles and pairs partition the triangle, and at 300K
nodes the sums over 8 shards equal the single-GPU gradient's repulsion and Z.

Which pairs a shard owns is restated here from the header's rule: positions
in blocks of T = 64 * tile_rows, row blocks a and nb-1-a form pair
min(a, nb-1-a), pair p goes to shard p mod n_shards, and a shard owns the
pairs {i, j} whose lower block is one of its row blocks."""
import numpy as np
import pytest

import oracle
from paper_2310_11186_amd import synth, tsgne

pytestmark = pytest.mark.gpu

F_TOL = 1e-5       # force sums, relative L2 (FP32 pair arithmetic)
Z_TOL = 1e-6       # Z partial, relative
F_TOL_FP32 = 1e-3  # all-FP32 mode
Z_TOL_FP32 = 1e-4


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def owned(n, R, shard, n_shards):
    T = 64 * R
    nb = -(-n // T)
    a = np.arange(nb)
    return (np.minimum(a, nb - 1 - a) % n_shards) == shard, np.arange(n) // T


def layout(n, seed, spread):
    rng = np.random.default_rng(seed)
    if spread == 0:
        return synth.initial_layout(n, seed)
    # a few clusters of different widths, as after the exaggeration phase
    c = rng.standard_normal((7, 2)) * spread
    k = rng.integers(0, 7, size=n)
    return (c[k] + rng.standard_normal((n, 2)) * (0.1 + rng.random(n)[:, None] * spread / 5)).astype(np.float32)


def run_shards(gpu, Y_np, n_shards, R, precision):
    import torch
    Y = torch.from_numpy(Y_np).to(gpu)
    out = []
    for s in range(n_shards):
        sh = tsgne.Shard(Y_np.shape[0], s, n_shards, R)
        info = sh.info()
        F, Z = sh.repulsion(Y, precision)
        out.append((info, F.cpu().numpy(), float(Z.cpu().numpy()[0])))
        sh.close()
    return out


@pytest.mark.parametrize("n,n_shards,R", [(1, 1, 4), (2, 3, 8), (700, 2, 4), (1000, 3, 4), (2500, 8, 4), (1000, 4, 1),
                                          (2500, 3, 8), (3001, 2, 15), (3001, 5, 0), (4200, 1, 16)])
@pytest.mark.parametrize("spread", [0, 8.0])
def test_shard_against_oracle(gpu, n, n_shards, R, spread):
    Y = layout(n, 40 + n, spread)
    res = run_shards(gpu, Y, n_shards, R, tsgne.TSGNE_PREC_SPLIT)
    Y64 = Y.astype(np.float64)
    tiles_total = pairs_total = 0
    F_sum = np.zeros((n, 2))
    Z_sum = 0.0
    for s, ((Rs, tiles, pairs), F, Z) in enumerate(res):
        if R:
            assert Rs == R
        counted, group = owned(n, Rs, s, n_shards)
        Fo, Zo = oracle.repulsion_terms(Y64, group=group, counted=counted.astype(np.uint8))
        if tiles == 0:
            assert pairs == 0 and Z == 0.0 and not F.any()
        else:
            assert rel_l2(F, Fo) <= F_TOL, (s, rel_l2(F, Fo))
            assert Z == pytest.approx(Zo, rel=Z_TOL, abs=1e-300)
        # block b is touched only by tiles (a, b), a <= b, of owned row blocks a:
        # rows of untouched blocks get exact zeros
        T = 64 * Rs
        for b in range(counted.shape[0]):
            if not counted[:b + 1].any():
                assert not F[b * T:(b + 1) * T].any()
        tiles_total += tiles
        pairs_total += pairs
        F_sum += F
        Z_sum += Z
    nb = -(-n // (64 * res[0][0][0]))
    assert tiles_total == nb * (nb + 1) // 2
    assert pairs_total == n * (n - 1)
    Fo, Zo = oracle.repulsion_terms(Y64)
    if n > 1:
        assert rel_l2(F_sum, Fo) <= F_TOL
        assert Z_sum == pytest.approx(Zo, rel=Z_TOL)


@pytest.mark.parametrize("n,n_shards,R", [(2500, 3, 8), (3001, 2, 15)])
def test_shard_fp32_mode(gpu, n, n_shards, R):
    Y = layout(n, 7, 8.0)
    for s, ((Rs, tiles, _), F, Z) in enumerate(run_shards(gpu, Y, n_shards, R, tsgne.TSGNE_PREC_FP32)):
        counted, group = owned(n, Rs, s, n_shards)
        Fo, Zo = oracle.repulsion_terms(Y.astype(np.float64), group=group, counted=counted.astype(np.uint8))
        assert rel_l2(F, Fo) <= F_TOL_FP32
        assert Z == pytest.approx(Zo, rel=Z_TOL_FP32)


def test_shard_repeated_calls_are_identical(gpu):
    import torch
    n = 3001
    Y = torch.from_numpy(layout(n, 3, 8.0)).to(gpu)
    sh = tsgne.Shard(n, 1, 3, 4)
    F1, Z1 = sh.repulsion(Y)
    F1, Z1 = F1.clone(), Z1.clone()
    sh.set_timing(True)
    F2, Z2 = sh.repulsion(Y)
    F3, Z3 = sh.repulsion(Y)
    ms, launches = sh.timing()
    assert torch.equal(F1, F2) and torch.equal(Z1, Z2) and torch.equal(F1, F3) and torch.equal(Z1, Z3)
    assert launches == 2 and ms > 0.0
    sh.close()


def test_shard_rejects_bad_arguments(gpu):
    import torch
    for args in [(0, 0, 1, 0), (10, 1, 1, 0), (10, -1, 2, 0), (10, 0, 0, 0), (10, 0, 1, 5), (10, 0, 70000, 0)]:
        with pytest.raises(tsgne.TsgneError) as e:
            tsgne.Shard(*args)
        assert e.value.status == tsgne.TSGNE_E_INVAL
    sh = tsgne.Shard(100, 0, 2, 4)
    Y = torch.zeros((100, 2), dtype=torch.float32, device=gpu)
    F = torch.empty((100, 2), dtype=torch.float64, device=gpu)
    Z = torch.empty(1, dtype=torch.float64, device=gpu)
    with pytest.raises(tsgne.TsgneError) as e:
        tsgne._check(tsgne.lib().tsgne_shard_repulsion(sh.handle, tsgne._ptr(Y), 7, tsgne._ptr(F), tsgne._ptr(Z),
                                                       None))
    assert e.value.status == tsgne.TSGNE_E_INVAL
    with pytest.raises(tsgne.TsgneError):
        tsgne._check(tsgne.lib().tsgne_shard_repulsion(sh.handle, None, 0, tsgne._ptr(F), tsgne._ptr(Z), None))
    sh.close()


def test_shards_at_300k_sum_to_the_single_gpu_repulsion(gpu):
    """8 shards of a 300,000-node layout (the size of the benchmark graph): the
    sum of their Z partials equals the single-GPU Z with the same tile, their
    force sums give the single-GPU gradient of a graph with no edges
    (g = -4 F / Z), and sampled rows of every shard match the oracle."""
    import torch
    n, G = 300_000, 8
    Y_np = layout(n, 5, 30.0)
    Y = torch.from_numpy(Y_np).to(gpu)
    shards = [tsgne.Shard(n, s, G, 0) for s in range(G)]
    R = shards[0].info()[0]
    F_sum = torch.zeros((n, 2), dtype=torch.float64, device=gpu)
    Z_sum = 0.0
    rng = np.random.default_rng(9)
    rows = np.unique(np.concatenate([rng.integers(0, n, 40), [0, n - 1, n // 2]])).astype(np.int32)
    Y64 = Y_np.astype(np.float64)
    for s, sh in enumerate(shards):
        assert sh.info()[0] == R
        F, Z = sh.repulsion(Y)
        F_sum += F
        Z_sum += float(Z.cpu().numpy()[0])
        counted, group = owned(n, R, s, G)
        Fo, _ = oracle.repulsion_terms(Y64, group=group, counted=counted.astype(np.uint8), rows=rows, with_Z=False)
        assert rel_l2(F.cpu().numpy()[rows], Fo) <= F_TOL
        sh.close()
    Fo, _ = oracle.repulsion_terms(Y64, rows=rows, with_Z=False)
    assert rel_l2(F_sum.cpu().numpy()[rows], Fo) <= F_TOL
    # the single-GPU path on a graph with no edges (gradient = repulsion only)
    rp = torch.zeros(n + 1, dtype=torch.int32, device=gpu)
    col = torch.zeros(0, dtype=torch.int32, device=gpu)
    X = torch.zeros((n, 1), dtype=torch.float32, device=gpu)
    g = tsgne.tsgne_build_P(rp, col, X, 30.0)
    params = tsgne.tsgne_params_default(tile_rows=R, repulsion=tsgne.TSGNE_REPULSION_SYMMETRIC)
    grad, Z1 = tsgne.tsgne_gradient(g, Y, 1.0, params)
    Z1 = float(Z1.cpu().numpy()[0])
    g.close()
    assert Z_sum == pytest.approx(Z1, rel=1e-12)
    assert rel_l2(-4.0 * F_sum.cpu().numpy() / Z_sum, grad.cpu().numpy()) <= 1e-6
