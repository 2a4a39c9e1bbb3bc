"""Pins of the keyframe-selection oracle (Sec. III-F, Eqs. (7)-(8)):
camera centres from known positions, the grid cell against exact rational
floor division, the candidate set by brute force, Eq. (7) on hand cases and
its limits, and the window rule by brute force."""
import itertools
from fractions import Fraction

import numpy as np

import scenegen
from oracle import chunks as oc
from oracle import keyframes as ok


def _cam_at(C, R=np.eye(3), z_near=0.2, z_far=50.0, f=100.0):
    C = np.asarray(C, np.float64)
    return scenegen.camera(R, -(np.asarray(R) @ C), f, f, 32.0, 24.0, 64, 48, z_near, z_far)


def test_position_is_the_camera_centre():
    # identity rotation: t = -C exactly, so the centre comes back exactly
    for C in ((0.0, 0.0, 0.0), (199.75, -3.5, 1.65), (-1e3, 2e3, -7.25)):
        assert (ok.position(_cam_at(C)) == np.asarray(C)).all()
    # rotated poses (look cameras) built from known centres
    for k, C in enumerate(((4.0, 4.0, 1.5), (-120.3, 455.9, 1.65))):
        cam = scenegen.look_camera(np.asarray(C), 0.3 + k, -0.1, 300, 300, 64, 48)
        assert np.allclose(ok.position(cam), C, rtol=0, atol=1e-12)


def test_grid_cell_hand_values_and_faces():
    g = 200.0
    below, above = np.nextafter(200.0, 0.0), np.nextafter(-200.0, 0.0)
    cases = {0.0: 0, 199.999: 0, 200.0: 1, 399.99999999999994: 1, 400.0: 2, -1e-9: -1,
             -200.0: -1, -200.00000000001: -2, -0.0: 0, 12345.0: 61,
             float(below): 0, float(above): -1, float(np.nextafter(600.0, 0.0)): 2}
    for p, c in cases.items():
        assert ok.grid_cell([p, p, p], g).tolist() == [c, c, c], p


def test_grid_cell_equals_exact_rational_floor():
    rng = np.random.default_rng(3)
    p = rng.uniform(-5000, 5000, (2000, 3))
    p[:50] = np.round(p[:50] / 200.0) * 200.0          # exactly on faces
    p[50:100] = np.nextafter(p[:50], -np.inf)           # just below them
    got = ok.grid_cell(p, 200.0)
    exp = np.array([[Fraction(float(x)) // 200 for x in row] for row in p], np.int64)
    assert (got == exp).all()


def test_candidate_set_by_brute_force():
    rng = np.random.default_rng(4)
    cent = rng.uniform(-600, 600, (80, 3))
    cent[::7] = np.round(cent[::7] / 200.0) * 200.0     # some keyframes on cell faces
    cams = [_cam_at(c) for c in cent]
    for latest in (0, 33, 79):
        got = ok.candidate_set(cams, latest, 200.0)
        ref = [Fraction(float(x)) // 200 for x in cent[latest]]
        exp = [[Fraction(float(x)) // 200 for x in c] == ref for c in cent]
        assert got.tolist() == exp
        assert got[latest]


def _grid_ids(side, offset):
    ax = np.arange(side) + offset
    cx, cy, cz = np.meshgrid(ax, ax, ax, indexing="ij")
    return np.sort(oc.encode_id(np.stack([cx.ravel(), cy.ravel(), cz.ravel()], 1)))


def test_overlap_of_a_frustum_inside_one_cell():
    s = 1.0
    ids = _grid_ids(5, -2)                               # cells -2..2 per axis
    c0 = oc.encode_id(np.array([[1, 0, -1]]))[0]
    # a short, narrow frustum around the centre of cell (1, 0, -1): it sees
    # that cell only
    cam = _cam_at((1.0, 0.0, -1.0), z_near=0.01, z_far=0.2, f=1000.0)
    r = ok.overlap([cam], ids, np.array([c0], np.uint64), s)
    assert r["n_visible"].tolist() == [1] and r["n_overlap"].tolist() == [1]
    assert r["overlap"].tolist() == [1.0]
    others = ids[ids != c0][:10]
    r = ok.overlap([cam], ids, others, s)
    assert r["n_visible"].tolist() == [1] and r["n_overlap"].tolist() == [0]
    assert r["overlap"].tolist() == [0.0]


def test_overlap_of_a_keyframe_that_sees_nothing_is_one():
    s = 1.0
    ids = _grid_ids(3, -1)                               # cells within [-1.5, 1.5]^3
    away = _cam_at((0.0, 0.0, 10.0), z_far=5.0)          # looks along +z from above them
    r = ok.overlap([away], ids, ids[:3], s)
    assert r["n_visible"].tolist() == [0] and r["overlap"].tolist() == [1.0]


def test_overlap_limits_and_monotonicity():
    s = 1.0
    ids = _grid_ids(6, -3)
    cams = scenegen.random_cameras(12, seed=5, extent=2.5)
    full = ok.overlap(cams, ids, ids, s)
    none = ok.overlap(cams, ids, np.array([], np.uint64), s)
    assert not full["tie"].any()
    seen = full["n_visible"] > 0
    assert seen.any()
    assert (full["overlap"] == 1.0).all()
    assert (none["overlap"][seen] == 0.0).all() and (none["overlap"][~seen] == 1.0).all()
    rng = np.random.default_rng(6)
    a = ids[rng.random(ids.size) < 0.3]
    b = np.union1d(a, ids[rng.random(ids.size) < 0.3])
    ra, rb = ok.overlap(cams, ids, a, s), ok.overlap(cams, ids, b, s)
    assert (ra["overlap"] <= rb["overlap"]).all()
    assert (ra["n_visible"] == full["n_visible"]).all()
    # Eq. (7) from the counts
    assert np.array_equal(ra["overlap"][seen], ra["n_overlap"][seen] / ra["n_visible"][seen])


def test_window_rule_by_brute_force():
    rng = np.random.default_rng(7)
    for trial in range(30):
        m = int(rng.integers(1, 9))
        in_set = rng.random(m) < 0.7
        ov = rng.choice([0.0, 0.25, 0.5, 1.0], m)        # ties on purpose
        n = int(rng.integers(1, 5))
        got = ok.window(in_set, ov, n)
        cand = [k for k in range(m) if in_set[k]]
        # brute force: among all subsets of the candidates of the window's
        # size, the chosen one is the greatest in (overlaps sorted
        # descending, then indices sorted descending)
        size = min(n, len(cand))
        best = max(itertools.combinations(cand, size),
                   key=lambda c: (sorted((ov[k] for k in c), reverse=True),
                                  sorted(c, reverse=True)))
        assert sorted(got.tolist()) == sorted(best)
        assert len(got) == size
