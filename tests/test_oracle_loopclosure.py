"""Pins of the loop-closure oracle (Sec. III-G)."""
import math

import numpy as np
from scipy.spatial.transform import Rotation

import scenegen
from oracle import chunks as oc
from oracle import loopclosure as olc


def _scene(n=6000, seed=3, drift=True):
    sc = scenegen.room_scene(n, seed=seed, sh_degree=0)
    P = sc["params"]
    ids = oc.encode_id(oc.chunk_coord(P[0:3].T, 2.0))
    order = np.lexsort((np.arange(P.shape[1]), ids))   # store order
    P, ids = P[:, order], ids[order]
    # optimisation has moved some means across a chunk face since they were
    # assigned: their stored chunk is not the one their mean lies in
    if drift:
        P[0, ::7] += np.float32(1.5)
    rng = np.random.default_rng(seed)
    m = rng.normal(size=P.shape).astype(np.float32)
    v = rng.uniform(size=P.shape).astype(np.float32)
    step = rng.integers(1, 50, P.shape[1]).astype(np.int32)
    return P, m, v, step, ids


def _cam(pos, yaw):
    return scenegen.look_camera(np.array(pos, float), yaw, 0.0, 300, 300, 320, 240, 0.2, 6.0)


def _rot_from_quat(q):
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def test_identity_correction_changes_nothing():
    P, m, v, step, ids = _scene(drift=False)
    out = olc.loop_closure(P, m, v, step, ids, 2.0, [(_cam((4, 4, 1.5), 0.3), np.eye(3), np.zeros(3))],
                           [])
    assert (out["params"] == P).all() and (out["m"] == m).all() and (out["step"] == step).all()
    assert (out["ids"] == ids).all()
    assert (out["owner"] >= 0).any()


def test_translation_by_one_chunk_moves_chunks_by_one():
    P, m, v, step, ids = _scene()
    kf = [(_cam((4, 4, 1.5), 0.3), np.eye(3), np.array([2.0, 0.0, 0.0]))]
    own = olc.assign(ids, 2.0, kf)
    out = olc.loop_closure(P, m, v, step, ids, 2.0, kf, [])
    moved = out["owner"] == 0
    assert moved.sum() == (own == 0).sum() > 100
    # the moved Gaussians, in their old store order, are the ones assigned
    old = P[:, own == 0]
    new_sorted = out["params"][:, moved]
    key = lambda A: np.lexsort(A[::-1])  # noqa: E731
    a = old.copy()
    a[0] = (a[0].astype(np.float64) + 2.0).astype(np.float32)
    assert (a[:, key(a)] == new_sorted[:, key(new_sorted)]).all()
    c_old = oc.chunk_coord(P[0:3, own == 0].T, 2.0)
    c_new = oc.chunk_coord(a[0:3].T, 2.0)
    assert (c_new[:, 0] == c_old[:, 0] + 1).all() and (c_new[:, 1:] == c_old[:, 1:]).all()


def test_rotation_composes_and_first_keyframe_wins():
    P, m, v, step, ids = _scene()
    R1 = Rotation.from_euler("z", 7, degrees=True).as_matrix()
    R2 = Rotation.from_euler("x", 11, degrees=True).as_matrix()
    kf = [(_cam((4, 4, 1.5), 0.0), R1, np.array([0.1, -0.2, 0.05])),
          (_cam((4, 4, 1.5), 0.4), R2, np.array([0.3, 0.0, 0.0]))]
    own = olc.assign(ids, 2.0, kf)
    both = set(oc.select_chunks([kf[0][0]], np.unique(ids), 2.0)["union_ids"].tolist())
    assert ((own == 0) == np.isin(ids, np.array(sorted(both), np.uint64))).all()
    assert (own == 1).any() and (own == -1).any()
    out = olc.loop_closure(P, m, v, step, ids, 2.0, kf, [])
    for k, R in ((0, R1), (1, R2)):
        sel_old = np.nonzero(own == k)[0][:20]
        for i in sel_old:
            q_old = P[6:10, i].astype(np.float64)
            j = np.nonzero((out["m"] == m[:, i:i + 1]).all(0))[0]
            assert j.size == 1
            q_new = out["params"][6:10, j[0]].astype(np.float64)
            mu_new = out["params"][0:3, j[0]].astype(np.float64)
            t = kf[k][2]
            mu_ref = R @ P[0:3, i].astype(np.float64) + t
            assert np.abs(mu_new - mu_ref).max() <= 2e-7 * max(1.0, np.abs(mu_ref).max())
            assert np.allclose(_rot_from_quat(q_new), R @ _rot_from_quat(q_old), atol=1e-6)
            assert abs(np.linalg.norm(q_new) - np.linalg.norm(q_old)) < 1e-5 * np.linalg.norm(q_old)


def test_regrouping_is_a_stable_sort_by_new_chunk():
    P, m, v, step, ids0 = _scene()
    kf = [(_cam((4, 4, 1.5), 0.3), Rotation.from_euler("z", 20, degrees=True).as_matrix(),
           np.array([0.7, 0.9, 0.0]))]
    out = olc.loop_closure(P, m, v, step, ids0, 2.0, kf, [])
    ids = out["ids"]
    assert (ids[1:] >= ids[:-1]).all()
    # within each chunk the m rows (unique per Gaussian) keep the old order
    pos_old = {tuple(m[:, i]): i for i in range(0, P.shape[1])}
    old_pos = np.array([pos_old[tuple(out["m"][:, j])] for j in range(P.shape[1])])
    old_ids = ids0
    for c in np.unique(ids):
        sel = np.nonzero(ids == c)[0]
        keys = list(zip(old_ids[old_pos[sel]], old_pos[sel]))
        assert keys == sorted(keys)
    assert (out["ids"] != old_ids[old_pos]).sum() > 10


def test_reset_touches_exactly_the_junction_chunks():
    P, m, v, step, ids = _scene()
    P[10, ::3] = -9.0                       # below the cap: kept
    # the correction moves part of the map into chunks that were empty before,
    # and the junction camera looks at them
    kf = [(_cam((4, 4, 1.5), 0.3), np.eye(3), np.array([20.0, 0.0, 0.0]))]
    jc = _cam((18, 6, 1.5), 0.3)
    out = olc.loop_closure(P, m, v, step, ids, 2.0, kf, [jc])
    vis = oc.select_chunks([jc], np.unique(out["ids"]), 2.0)["union_ids"]
    want = np.isin(out["ids"], vis)
    assert (out["reset"] == want).all() and want.any() and (~want).any()
    assert not np.isin(vis, ids).all()
    assert (out["m"][:, want] == 0).all() and (out["v"][:, want] == 0).all()
    assert (out["step"][want] == 0).all()
    lg = out["params"][10]
    assert (lg[want] <= np.float32(olc.LOGIT_CAP)).all()
    assert (lg[want] == -9.0).any() and (lg[want] == np.float32(olc.LOGIT_CAP)).any()
    # outside the junction chunks the opacity logits are the old ones
    keep = ~want
    assert np.array_equal(np.sort(lg[keep]), np.sort(P[10][_old_of(P, out, keep)]))
    assert abs(olc.LOGIT_CAP - math.log(0.01 / 0.99)) < 1e-15


def _old_of(P, out, sel):
    """Mask over the old store of the Gaussians at `sel` in the new one (the
    colour rows, untouched by the correction, identify a Gaussian)."""
    key = {tuple(P[11:, i]): i for i in range(P.shape[1])}
    mask = np.zeros(P.shape[1], bool)
    for j in np.nonzero(sel)[0]:
        mask[key[tuple(out["params"][11:, j])]] = True
    return mask


def test_only_the_correction_reassigns_chunks():
    P, m, v, step, ids = _scene()
    kf = [(_cam((4, 4, 1.5), 0.3), Rotation.from_euler("z", 5, degrees=True).as_matrix(),
           np.array([0.4, 0.0, 0.0]))]
    out = olc.loop_closure(P, m, v, step, ids, 2.0, kf, [])
    pos_old = {tuple(m[:, i]): i for i in range(P.shape[1])}
    src = np.array([pos_old[tuple(out["m"][:, j])] for j in range(P.shape[1])])
    untouched = out["owner"] < 0
    # untransformed Gaussians keep their stored chunk, drifted or not
    assert (out["ids"][untouched] == ids[src[untouched]]).all()
    drifted = ids != olc.store_ids(P, 2.0)
    assert (drifted[src[untouched]]).any()
    # transformed ones are in the chunk of their corrected mean
    moved = ~untouched
    assert (out["ids"][moved] == olc.store_ids(out["params"][:, moved], 2.0)).all()
