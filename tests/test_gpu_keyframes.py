"""GPU parity of keyframe selection (Sec. III-F, Eqs. (7)-(8)) through the
C ABI: candidate-set membership, visible and overlapping chunk counts and
the window bit-exact against the oracle."""
import numpy as np
import pytest
import torch

import scenegen
from oracle import chunks as oc
from oracle import keyframes as ok
from paper_2511_23030_amd import dcgs as D

pytestmark = pytest.mark.gpu


def _check(ctx, cams, latest, g, ids, active, s, n_window):
    ref = ok.overlap(cams, ids, active, s)
    assert not ref["tie"].any()
    in_set = ok.candidate_set(cams, latest, g)
    dev = torch.from_numpy(ids.view(np.int64)).cuda()
    got = ctx.keyframe_overlap(cams, latest, dev, s, active, grid=g, n_window=n_window)
    assert (got["in_set"].astype(bool) == in_set).all()
    assert (got["n_visible"] == ref["n_visible"]).all()
    assert (got["n_overlap"] == ref["n_overlap"]).all()
    assert np.array_equal(got["overlap"], ref["overlap"])      # same float64 division
    assert got["window"].tolist() == ok.window(in_set, ref["overlap"], n_window).tolist()
    return got


def test_keyframe_overlap_random_cameras(ctx):
    s = 1.0
    coords = scenegen.grid_coords(6, -3)
    ids = np.sort(oc.encode_id(coords))
    cams = scenegen.random_cameras(40, seed=81, extent=2.5)
    # a few keyframes exactly on faces of the 2 m keyframe grid and just below
    for k, C in ((3, (2.0, -2.0, 0.0)), (4, (np.nextafter(2.0, 0.0), -2.0, 0.0))):
        R = np.asarray(cams[k]["R"])
        cams[k] = scenegen.camera(R, -(R @ np.asarray(C)), cams[k]["fx"], cams[k]["fy"],
                                  cams[k]["cx"], cams[k]["cy"], cams[k]["width"],
                                  cams[k]["height"], cams[k]["z_near"], cams[k]["z_far"])
    rng = np.random.default_rng(82)
    active = ids[rng.random(ids.size) < 0.4]
    for latest in (39, 3, 4):
        got = _check(ctx, cams, latest, 2.0, ids, active, s, n_window=5)
        print(f"latest {latest}: {int(got['in_set'].sum())} candidates, window "
              f"{got['window'].tolist()}", flush=True)


def test_keyframe_overlap_on_the_driving_corridor(ctx):
    """Keyframes every 2 m along the corridor, 50 m chunks, the paper's
    200 m keyframe grid, the chunks of the last keyframes as the resident
    set."""
    s = 50.0
    path = scenegen.driving_path(20)
    cams = scenegen.driving_trajectory(path, 240, z_far=350.0)[::4]
    # every chunk cell along the corridor (road and facades, one z layer)
    cells = np.unique(oc.chunk_coord(np.c_[path, np.zeros(len(path))], s), axis=0)
    near = np.concatenate([cells + np.array([dx, dy, 0]) for dx in (-1, 0, 1)
                           for dy in (-1, 0, 1)])
    ids = np.unique(oc.encode_id(near))
    sel = oc.select_chunks(cams[-3:], ids, s)
    active = sel["union_ids"]
    got = _check(ctx, cams, len(cams) - 1, 200.0, ids, active, s, n_window=16)
    assert got["in_set"].sum() >= 16
    assert (got["overlap"][-3:] == 1.0).all()        # their chunks are the active set
