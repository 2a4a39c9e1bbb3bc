"""GPU parity of chunk IDs (Eqs. 5-6) and visible-chunk selection."""
import numpy as np
import pytest
import torch

import scenegen
from oracle import chunks as oc
from paper_2511_23030_amd import dcgs as D

pytestmark = pytest.mark.gpu


def test_chunk_ids_bit_exact(ctx):
    rng = np.random.default_rng(1)
    s = 2.0
    mean = rng.uniform(-5000, 5000, (3, 100_000)).astype(np.float32)
    # faces of cells (exact in float32), negatives, and their float32 neighbours
    faces = np.array([1.0, 3.0, -1.0, -3.0, 0.0, 999.0], np.float32)
    mean[0, :6] = faces
    mean[1, 6:12] = np.nextafter(faces, np.float32(-np.inf))
    mean[2, 12:18] = np.nextafter(faces, np.float32(np.inf))
    t = torch.from_numpy(mean).cuda()
    got = ctx.chunk_ids(t, s).cpu().numpy().view(np.uint64)
    exp = oc.encode_id(oc.chunk_coord(mean.T, s))
    assert (got == exp).all()


def test_chunk_ids_range_error(ctx):
    mean = torch.zeros(3, 10, device="cuda")
    mean[1, 3] = 1e9                 # coordinate 5e8 >> 2^20 at s = 2
    with pytest.raises(D.DcgsError) as e:
        ctx.chunk_ids(mean, 2.0)
    assert e.value.status == 6


@pytest.mark.parametrize("n_views", [1, 16])
def test_select_matches_exact_visibility(ctx, n_views):
    s = 1.0
    coords = scenegen.grid_coords(8, -4)
    ids = np.sort(oc.encode_id(coords))
    cams = scenegen.random_cameras(n_views, seed=40 + n_views, extent=3.0)
    ref = oc.select_chunks(cams, ids, s)
    assert not ref["tie"].any()
    dev_ids = torch.from_numpy(ids.view(np.int64)).cuda()
    out_ids, out_mask, count = ctx.select_chunks(cams, dev_ids, s)
    k = int(count.item())
    assert k == ref["union_ids"].size
    assert (out_ids[:k].cpu().numpy().view(np.uint64) == ref["union_ids"]).all()
    assert (out_mask[:k].cpu().numpy().view(np.uint16) == ref["view_mask"]).all()


def test_select_room_trajectory(ctx):
    """The indoor workload: every chunk of the room against 50 poses."""
    sc = scenegen.room_scene(20_000, seed=10, sh_degree=0)
    s = 2.0
    ids = np.unique(oc.encode_id(oc.chunk_coord(sc["params"][0:3].T, s)))
    cams = scenegen.room_trajectory(50, seed=11, z_far=6.0)
    dev_ids = torch.from_numpy(ids.view(np.int64)).cuda()
    for cam in cams[::5]:
        ref = oc.select_chunks([cam], ids, s)
        assert not ref["tie"].any()
        out_ids, _, count = ctx.select_chunks([cam], dev_ids, s)
        k = int(count.item())
        assert (out_ids[:k].cpu().numpy().view(np.uint64) == ref["union_ids"]).all()
