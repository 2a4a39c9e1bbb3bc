"""Keyframe selection (Sec. III-F): the spatial candidate set, the overlap
metric and the usage/loss rule, checked by brute force on small cases."""
import math

import numpy as np

from paper_2511_23030_amd import schedule as S


def test_grid_cell_is_elementwise_floor():
    assert S.grid_cell((0.0, 0.0, 0.0)) == (0, 0, 0)
    assert S.grid_cell((199.999, 200.0, -0.001)) == (0, 1, -1)
    assert S.grid_cell((-400.0, 401.0, 5.0), 200.0) == (-2, 2, 0)


def test_overlap_definition():
    assert S.overlap({1, 2, 3, 4}, {2, 4, 9}) == 0.5
    assert S.overlap(set(), {1}) == 1.0
    assert S.overlap({7}, set()) == 0.0


def test_candidates_are_exactly_the_latest_cell():
    rng = np.random.default_rng(0)
    sch = S.KeyframeScheduler(grid=200.0)
    pos = rng.uniform(-500, 500, size=(60, 3))
    for k, p in enumerate(pos):
        sch.add(k, p, [k])
    cell = tuple(np.floor(pos[-1] / 200.0).astype(int))
    brute = [k for k in range(60) if tuple(np.floor(pos[k] / 200.0).astype(int)) == cell]
    assert sch.candidates() == brute


def test_selection_spends_uses_and_favours_high_loss():
    sch = S.KeyframeScheduler(grid=200.0, usage=2)
    for k in range(5):
        sch.add(k, (10.0 * k, 0.0, 0.0), {k, k + 1})
    losses = {0: 0.1, 1: 0.5, 2: 0.3, 3: 0.9, 4: 0.2}
    for k, v in losses.items():
        sch.report_loss(k, v)
    first = sch.select(2)
    assert first == [3, 1]
    seen = []
    while any(sch.left[k] > 0 for k in range(5)):
        seen += sch.select(2)
    # every keyframe is used twice before any gets more uses, high loss first
    assert sorted(first + seen) == sorted([0, 1, 2, 3, 4] * 2)
    assert seen[:4] == [3, 1, 2, 4]
    # out of uses: the high-loss half gets `usage` more, the rest one
    sch.select(5)
    assert sch.left[3] == 1 and sch.left[1] == 1 and sch.left[2] == 1
    assert sch.left[0] == 0 and sch.left[4] == 0


def test_overlap_breaks_ties_between_equal_losses():
    sch = S.KeyframeScheduler()
    sch.add("a", (0, 0, 0), {1, 2})
    sch.add("b", (1, 0, 0), {3, 4})
    assert math.isinf(sch.loss["a"])
    assert sch.select(1, active_chunks={3, 4}) == ["b"]
