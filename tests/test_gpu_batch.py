"""Batched optimisation (tsgne_batch_run) and the tile autotuner, through the
C-ABI.  A graph advanced inside a batch must equal the same graph run alone
with the same tile size, bit for bit; the batch replays a captured step many
times between eager work, and every graph is checked after it."""
import numpy as np
import pytest

import oracle
from paper_2310_11186_amd import synth, tsgne

pytestmark = pytest.mark.gpu


def upload(gi, gpu):
    import torch
    rp, col = tsgne.tsgne_csr_from_edges(gi.n, gi.edges)
    g = tsgne.tsgne_build_P(torch.from_numpy(rp).to(gpu), torch.from_numpy(col).to(gpu),
                            torch.from_numpy(gi.X).to(gpu), 30.0)
    return g


def small_batch(seed=0):
    sizes = [300, 700, 1500, 2600, 257, 1031]
    return [synth.small_sbm(n, 3, 5.0, 8, seed * 100 + k) for k, n in enumerate(sizes)]


@pytest.mark.parametrize("R", [1, 2, 4, 8, 12, 16])
def test_batch_equals_alone_bitwise(gpu, R):
    import torch
    gis = small_batch(1)
    graphs = [upload(gi, gpu) for gi in gis]
    n_iter = [60, 35, 51, 60, 7, 26]
    p = tsgne.tsgne_params_default(exaggeration_iters=20, learning_rate=40.0, tile_rows=R,
                                   repulsion=tsgne.TSGNE_REPULSION_SYMMETRIC)
    Ys = [torch.from_numpy(gi.Y0).to(gpu) for gi in gis]
    tsgne.tsgne_batch_run(graphs, Ys, n_iter, p)
    for gi, g, Yb, k in zip(gis, graphs, Ys, n_iter):
        Ya = torch.from_numpy(gi.Y0).to(gpu)
        tsgne.tsgne_run(g, Ya, k, p)
        torch.cuda.synchronize()
        assert torch.equal(Ya, Yb), gi.n


def test_batch_matches_oracle(gpu):
    import torch
    gis = small_batch(2)[:3]
    graphs = [upload(gi, gpu) for gi in gis]
    p = tsgne.tsgne_params_default(exaggeration_iters=10, learning_rate=40.0)
    Ys = [torch.from_numpy(gi.Y0).to(gpu) for gi in gis]
    tsgne.tsgne_batch_run(graphs, Ys, [20, 20, 20], p)
    for gi, Y in zip(gis, Ys):
        rp, col = oracle.csr_from_edges(gi.n, gi.edges)
        P, _ = oracle.build_P(rp, col, gi.X, 30.0)
        oY, _, _, _ = oracle.run(rp, col, P, gi.Y0, n_steps=20, exaggeration_iters=10, eta=40.0)
        err = np.linalg.norm(Y.cpu().numpy() - oY) / np.linalg.norm(oY)
        assert err <= 1e-4, (gi.n, err)


def test_autotune_picks_a_tile_and_leaves_inputs(gpu):
    import torch
    gis = small_batch(3)
    graphs = [upload(gi, gpu) for gi in gis]
    Ys = [torch.from_numpy(gi.Y0).to(gpu) for gi in gis]
    before = [Y.clone() for Y in Ys]
    best, ms = tsgne.tsgne_autotune(graphs, Ys, tsgne.tsgne_params_default(), steps=2)
    assert best in tsgne.AUTOTUNE_TILES and len(ms) == len(tsgne.AUTOTUNE_TILES)
    assert all(m > 0 for m in ms) and ms[tsgne.AUTOTUNE_TILES.index(best)] == min(ms)
    for a, b in zip(Ys, before):
        assert torch.equal(a, b)


def test_batch_rejects_bad_arguments(gpu):
    import torch
    gi = synth.small_sbm(400, 2, 4.0, 4, 9)
    g = upload(gi, gpu)
    Y = torch.from_numpy(gi.Y0).to(gpu)
    p = tsgne.tsgne_params_default()
    with pytest.raises(tsgne.TsgneError) as e:
        tsgne.tsgne_batch_run([g, g], [Y, Y.clone()], [5, 5], p)
    assert e.value.status == tsgne.TSGNE_E_INVAL
    with pytest.raises(tsgne.TsgneError):
        tsgne.tsgne_batch_run([g], [Y], [-1], p)


def test_full_batch_workload_sampled(gpu):
    """The benchmark's whole batch (256 graphs, 2.94M nodes) in its own launch
    configuration (the autotuner's tile): 8 batched steps, then the smallest,
    a middle and the largest graph run alone with the same tile must end
    bitwise equal, and the smallest matches the FP64 oracle."""
    import torch
    gis = synth.batch_workload()
    graphs = [upload(gi, gpu) for gi in gis]
    steps = 8
    params = tsgne.tsgne_params_default(exaggeration_iters=187)
    Y0 = [torch.from_numpy(gi.Y0).to(gpu) for gi in gis]
    best, _ = tsgne.tsgne_autotune(graphs, Y0, params, steps=2)
    p = tsgne.tsgne_params_default(exaggeration_iters=187, tile_rows=best)
    Yb = [y.clone() for y in Y0]
    tsgne.tsgne_batch_run(graphs, Yb, [steps] * len(gis), p)
    order = sorted(range(len(gis)), key=lambda k: gis[k].n)
    for k in (order[0], order[len(order) // 2], order[-1]):
        Ya = Y0[k].clone()
        tsgne.tsgne_run(graphs[k], Ya, steps, tsgne.tsgne_params_default(
            exaggeration_iters=187, tile_rows=best, repulsion=tsgne.TSGNE_REPULSION_SYMMETRIC))
        torch.cuda.synchronize()
        assert torch.equal(Ya, Yb[k]), gis[k].n
    k = order[0]
    gi = gis[k]
    rp, col = oracle.csr_from_edges(gi.n, gi.edges)
    P, _ = oracle.build_P(rp, col, gi.X, 30.0)
    eta = float(np.float32(max(np.float32(gi.n) / np.float32(48.0), np.float32(50.0))))   # the automatic rate
    oY, _, _, _ = oracle.run(rp, col, P, gi.Y0, n_steps=steps, exaggeration_iters=187, eta=eta)
    err = np.linalg.norm(Yb[k].cpu().numpy() - oY) / np.linalg.norm(oY)
    assert err <= 1e-4, (gi.n, err)
    for g in graphs:
        g.close()


def test_batch_with_per_graph_tiles_equals_alone_bitwise(gpu):
    """Graphs of one batch with different tiles (explicit, and 0 = each
    graph's single-graph plan): the tile groups run side by side, and every
    graph equals its own tsgne_run with its tile, bit for bit."""
    import torch
    gis = small_batch(3) + [synth.small_sbm(n, 4, 6.0, 8, 390 + k) for k, n in enumerate([12_500, 5200])]
    graphs = [upload(gi, gpu) for gi in gis]
    n_iter = [60, 35, 51, 60, 7, 26, 40, 31]
    tiles = [1, 2, 4, 8, 12, 16, 0, 0]
    p = tsgne.tsgne_params_default(exaggeration_iters=20, learning_rate=40.0,
                                   repulsion=tsgne.TSGNE_REPULSION_SYMMETRIC)
    Ys = [torch.from_numpy(gi.Y0).to(gpu) for gi in gis]
    tsgne.tsgne_batch_run_tiles(graphs, Ys, n_iter, tiles, p)
    for gi, g, Yb, k, R in zip(gis, graphs, Ys, n_iter, tiles):
        Ya = torch.from_numpy(gi.Y0).to(gpu)
        pa = tsgne.tsgne_params_default(exaggeration_iters=20, learning_rate=40.0, tile_rows=R,
                                        repulsion=tsgne.TSGNE_REPULSION_SYMMETRIC)
        tsgne.tsgne_run(g, Ya, k, pa)
        torch.cuda.synchronize()
        assert torch.equal(Ya, Yb), (gi.n, R)
    with pytest.raises(tsgne.TsgneError) as e:
        tsgne.tsgne_batch_run_tiles(graphs, Ys, n_iter, [3] + tiles[1:], p)
    assert e.value.status == tsgne.TSGNE_E_INVAL


def test_autotune_tiles_by_bucket_and_cache(gpu, tmp_path):
    """The bucket autotuner returns one supported tile per size bucket, leaves
    the layouts alone, writes its choices to the cache under this device's
    architecture, and takes cached buckets as given on the next call; the
    tuned batch equals the graphs run alone with those tiles."""
    import json
    import math

    import torch
    gis = small_batch(4) + [synth.small_sbm(n, 4, 6.0, 8, 400 + k) for k, n in enumerate([9000, 17_000])]
    graphs = [upload(gi, gpu) for gi in gis]
    p = tsgne.tsgne_params_default(exaggeration_iters=20, learning_rate=40.0)
    Ys = [torch.from_numpy(gi.Y0).to(gpu) for gi in gis]
    before = [Y.clone() for Y in Ys]
    cache = str(tmp_path / "tiles.json")
    tiles, ms_u, ms_t = tsgne.tsgne_autotune_tiles(graphs, Ys, p, steps=2, cache_path=cache)
    assert all(torch.equal(a, b) for a, b in zip(Ys, before))
    assert all(t in (2, 4, 8, 12, 16) for t in tiles)
    bucket = [int(math.floor(math.log2(gi.n))) for gi in gis]
    for b in set(bucket):
        assert len({t for t, bb in zip(tiles, bucket) if bb == b}) == 1
    assert 0 < ms_t <= ms_u
    saved = json.load(open(cache))
    assert len(saved) == 1
    arch, table = next(iter(saved.items()))
    assert arch.startswith("gfx")
    assert {int(k): v for k, v in table.items()} == {b: t for b, t in zip(bucket, tiles)}
    # the cache fixes every bucket now: rewrite it to other tiles and they are used
    forced = {str(b): 4 for b in set(bucket)}
    json.dump({arch: forced, "gfx000": {"3": 8}}, open(cache, "w"))
    tiles2, _, _ = tsgne.tsgne_autotune_tiles(graphs, Ys, p, steps=1, cache_path=cache)
    assert tiles2 == [4] * len(gis)
    assert json.load(open(cache))["gfx000"] == {"3": 8}
    n_iter = [30] * len(gis)
    tsgne.tsgne_batch_run_tiles(graphs, Ys, n_iter, tiles, p)
    for gi, g, Yb, R in zip(gis, graphs, Ys, tiles):
        Ya = torch.from_numpy(gi.Y0).to(gpu)
        pa = tsgne.tsgne_params_default(exaggeration_iters=20, learning_rate=40.0, tile_rows=R,
                                        repulsion=tsgne.TSGNE_REPULSION_SYMMETRIC)
        tsgne.tsgne_run(g, Ya, 30, pa)
        torch.cuda.synchronize()
        assert torch.equal(Ya, Yb), (gi.n, R)
