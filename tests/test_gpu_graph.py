"""The graph-captured mapping window against the eager batched window: every
replay's images, loss and the pool state after it are bit-identical, also
when a window overflows its pair capacity and is run again after a
rebuild."""
import numpy as np
import pytest
import torch

import scenegen
from paper_2511_23030_amd import dcgs as D
from paper_2511_23030_amd import mapping

pytestmark = pytest.mark.gpu

W, H, F = 320, 180, 160.0


@pytest.fixture(scope="module")
def room():
    sc = scenegen.room_scene(300_000, seed=10, sh_degree=3)
    cams = scenegen.room_trajectory(240, seed=11, width=W, height=H, focal=F, z_far=5.0)
    return scenegen.perturb(sc["params"], seed=12), cams


def _loop(ctx, params, V, **loss):
    pool = D.Pool(ctx, 3, budget=10**9)
    pool.ingest(params, 2.0)
    loop = mapping.MappingLoop(ctx, pool, 3, 2.0, 320_000, W, H, (16, 16), ppt=2, **loss)
    loop._window_buffers(V)
    return pool, loop


def _windows(cams, V, k):
    return [cams[5 + w * V * 3: 5 + (w + 1) * V * 3: 3] for w in range(k)]


def _targets(V, seed):
    return torch.from_numpy(np.stack([scenegen.target_image(W, H, seed=seed + v)
                                      for v in range(V)])).cuda()


def _compare_pools(pool_a, pool_b):
    ids, counts = pool_a.chunks()
    for cid, c in zip(ids, counts):
        for x, y in zip(pool_a.read_chunk(cid, c), pool_b.read_chunk(cid, c)):
            assert (x == y).all(), cid


@pytest.mark.parametrize("V", [1, 8])
def test_graph_replays_match_eager(ctx, room, V):
    params, cams = room
    wins = _windows(cams, V, 4)
    pool_a, loop_a = _loop(ctx, params, V)
    pool_b, loop_b = _loop(ctx, params, V)
    loop_b.build_graph(V, pair_capacity=4_000_000)
    for w, cw in enumerate(wins):
        tg = _targets(V, 100 + w)
        print(f"case graph V={V} window {w}", flush=True)
        loop_a.window_step(cw, tg)
        loop_b.window_step_graph(cw, tg)
        loop_b.sync_graph()
        torch.cuda.synchronize()
        assert torch.equal(loop_a.rgb_v, loop_b.rgb_v)
        assert torch.equal(loop_a.depth_v, loop_b.depth_v)
        assert torch.equal(loop_a.stats, loop_b.stats)
        assert loop_a.last["n_active"] == loop_b.last["n_active"]
        assert loop_b.win.pairs() == loop_a.state.info()["n_pairs"]
    _compare_pools(pool_a, pool_b)
    # the same window replayed twice more, eager work in between
    for rep in range(2):
        tg = _targets(V, 200 + rep)
        loop_a.window_step(wins[1], tg)
        loop_b.window_step_graph(wins[1], tg)
        loop_b.sync_graph()
        assert torch.equal(loop_a.rgb_v, loop_b.rgb_v)
    _compare_pools(pool_a, pool_b)
    loop_b.win.close()
    pool_a.close()
    pool_b.close()


def test_graph_overflow_is_redone_in_order(ctx, room):
    params, cams = room
    V = 4
    wins = _windows(cams, V, 4)
    pool_a, loop_a = _loop(ctx, params, V)
    pool_b, loop_b = _loop(ctx, params, V)
    loop_b.build_graph(V, pair_capacity=2000)      # far too small: every window overflows
    for w, cw in enumerate(wins):
        tg = _targets(V, 300 + w)
        loop_a.window_step(cw, tg)
        loop_b.window_step_graph(cw, tg)           # overflow is found two launches later
    loop_b.sync_graph()
    torch.cuda.synchronize()
    assert loop_b.win_pairs > 2000
    assert torch.equal(loop_a.rgb_v, loop_b.rgb_v)
    _compare_pools(pool_a, pool_b)
    loop_b.win.close()
    pool_a.close()
    pool_b.close()


def test_graph_full_loss_matches_eager(ctx, room):
    """The full mapping loss (SSIM, lambda_s = 0.2, and depth L1, lambda_depth
    = 0.1) inside the graph: images, the four loss sums and the pool after
    every window equal the eager batched window bit for bit."""
    params, cams = room
    V = 4
    wins = _windows(cams, V, 3)
    loss = dict(lambda_s=0.2, lambda_depth=0.1)
    pool_a, loop_a = _loop(ctx, params, V, **loss)
    pool_b, loop_b = _loop(ctx, params, V, **loss)
    loop_b.build_graph(V, pair_capacity=4_000_000)
    for w, cw in enumerate(wins):
        tg = _targets(V, 400 + w)
        td = torch.from_numpy(scenegen.target_image(W, H, seed=500 + w, channels=V) * 4.0).cuda()
        print(f"case graph full loss window {w}", flush=True)
        loop_a.window_step(cw, tg, target_depths=td)
        loop_b.window_step_graph(cw, tg, target_depths=td)
        loop_b.sync_graph()
        torch.cuda.synchronize()
        assert torch.equal(loop_a.rgb_v, loop_b.rgb_v)
        assert torch.equal(loop_a.depth_v, loop_b.depth_v)
        assert torch.equal(loop_a.stats, loop_b.stats)
        assert float(loop_b.stats[2]) > 0 and float(loop_b.stats[3]) > 0
    _compare_pools(pool_a, pool_b)
    with pytest.raises(ValueError):
        loop_b.window_step_graph(wins[0], _targets(V, 600))
    loop_b.win.close()
    pool_a.close()
    pool_b.close()
