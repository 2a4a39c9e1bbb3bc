"""Oracle: keyframe selection of Sec. III-F ("Keyframe Selection").

TEST INFRASTRUCTURE ONLY (see the package header).

Functions and what pins them (tests/test_oracle_keyframes.py):

* ``position``       A keyframe's 3D position p_k: its camera centre
                     -R^T t, in float64 with each product and sum rounded
                     in order.  Pinned by cameras built from known centres.
* ``grid_cell``      The discretisation of Eq. (8): floor(p / g) per axis
                     (g = 200 m), exact (not the floor of the rounded float64
                     quotient, which differs just below a cell face).  Pinned
                     by hand values on and next to cell faces and by exact
                     rational floor division.
* ``candidate_set``  K(p) of Eq. (8): the keyframes whose grid cell equals
                     that of p; the selection step takes p = the position of
                     the most recently added keyframe.  Pinned by brute force
                     with exact rational arithmetic.
* ``overlap``        Eq. (7): |C_v(k) & C_active| / |C_v(k)|, C_v(k) the
                     chunks keyframe k sees (the exact visibility of
                     ``chunks.select_chunks``) and C_active the resident
                     chunks.  A keyframe that sees no chunk needs nothing
                     loaded: its overlap is read as 1.  Pinned by hand cases
                     (a frustum inside one cell), the all-resident and
                     none-resident limits, and monotonicity in C_active.
* ``window``         Window formation for batched mapping (this library's
                     reading; the paper picks keyframes inside K(p_latest)
                     with CaRtGS's usage rule, which is not built): the n
                     keyframes of K(p_latest) with the highest overlap, ties
                     to the more recent keyframe.  Pinned by brute force over
                     all subsets on small cases.
"""
from __future__ import annotations

import numpy as np

from . import chunks as oc


def position(cam: dict) -> np.ndarray:
    """Camera centre C = -R^T t of a world-to-camera pose (float64)."""
    R = np.asarray(cam["R"], np.float64).reshape(3, 3)
    t = np.asarray(cam["t"], np.float64).reshape(3)
    C = np.empty(3, np.float64)
    for i in range(3):
        C[i] = -((R[0, i] * t[0] + R[1, i] * t[1]) + R[2, i] * t[2])
    return C


def grid_cell(p, g: float) -> np.ndarray:
    """floor(p / g) per axis (int64), exact: the float64 quotient can round
    up to an integer when p lies just below a cell face, so the estimate is
    corrected until k g <= p < (k + 1) g holds (k g is exact in float64 for
    the cell numbers that occur)."""
    p = np.asarray(p, np.float64)
    g = float(g)
    k = np.floor(p / g)
    k = np.where(k * g > p, k - 1.0, k)
    k = np.where((k + 1.0) * g <= p, k + 1.0, k)
    return k.astype(np.int64)


def candidate_set(cams: list, latest: int, g: float) -> np.ndarray:
    """Eq. (8): in_set[k] = (cell of keyframe k == cell of keyframe latest)."""
    ref = grid_cell(position(cams[latest]), g)
    return np.array([bool((grid_cell(position(c), g) == ref).all()) for c in cams])


def overlap(cams: list, ids: np.ndarray, active_ids: np.ndarray, s: float) -> dict:
    """Eq. (7) for every keyframe.  Returns n_visible, n_overlap (int64),
    overlap (float64) and tie (a chunk of that keyframe touches its frustum
    within rounding distance: excluded from bit-exact comparison)."""
    ids = np.asarray(ids, np.uint64)
    act = np.isin(ids, np.asarray(active_ids, np.uint64))
    sel = oc.select_chunks(cams, ids, s)
    vis = sel["visible"]
    n_vis = vis.sum(axis=1).astype(np.int64)
    n_ov = (vis & act[None, :]).sum(axis=1).astype(np.int64)
    ov = np.where(n_vis > 0, n_ov / np.maximum(n_vis, 1), 1.0)
    return dict(n_visible=n_vis, n_overlap=n_ov, overlap=ov.astype(np.float64),
                tie=sel["tie"].any(axis=1))


def window(in_set: np.ndarray, ov: np.ndarray, n: int) -> np.ndarray:
    """The n keyframes of the candidate set with the highest overlap, ties to
    the higher (more recent) index; fewer when the set is smaller."""
    cand = [k for k in range(len(in_set)) if in_set[k]]
    cand.sort(key=lambda k: (-ov[k], -k))
    return np.array(cand[:n], np.int64)
