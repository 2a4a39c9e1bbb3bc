"""Oracle: loop-closure correction of a chunked Gaussian map (Sec. III-G
"Cross-Chunk Transformation", "Chunk Redistribution", "Post-Correction
Refinement"), in float64 on float32 inputs.

TEST INFRASTRUCTURE ONLY (see the package header).

Readings (the paper describes the steps, not their arithmetic):

* affected keyframes come in order, each with a rigid correction (R, t)
  mapping old world coordinates to corrected ones;
* a keyframe's correction applies to every Gaussian of every chunk the
  exact visibility test of Sec. III-D selects for its camera; a chunk
  selected by several affected keyframes takes the first one's correction
  (the global transformation mask: no Gaussian is transformed twice);
* a transformed Gaussian's mean becomes R mean + t and its (unnormalised)
  rotation quaternion q = (w, x, y, z) becomes q_R (x) q (Hamilton product),
  q_R the unit quaternion of R with w >= 0; scales, opacity and colour
  coefficients are unchanged, and so are its Adam moments and step count;
* redistribution: a transformed Gaussian's chunk is recomputed (Eq. 5)
  from its corrected float32 mean; every other Gaussian stays in the chunk
  the store holds it in (optimisation may have moved its mean across a
  chunk face: only the correction reassigns); the store is regrouped by
  chunk in ascending EncodedID, keeping the previous order (ascending old
  EncodedID, then stored order) among the Gaussians of a chunk;
* refinement reset, after redistribution: for every Gaussian of the chunks
  a junction camera selects, the opacity logit becomes min(logit,
  logit(0.01)), its Adam moments 0 and its step count 0.

The store is the flat [R][N] parameter array (and moments [R][N], steps
[N]) with the EncodedID of the chunk holding each Gaussian [N], in store
order: ascending EncodedID, stored order inside a chunk.

What pins each function (tests/test_oracle_loopclosure.py): the identity
correction changes nothing; a pure translation by one chunk side shifts
every transformed Gaussian's chunk coordinate by one; the rotation matrix
of the corrected quaternion equals R times the old rotation (textbook
quaternion-to-matrix formula); overlapping keyframes apply the first
correction only; the regrouped order against a brute-force stable sort;
the reset touches exactly the junction chunks; an untransformed Gaussian
whose mean left its chunk stays there.
"""
from __future__ import annotations

import math

import numpy as np

from . import chunks as oc
from .prefetch import quat_wxyz

ROW_MEAN, ROW_QUAT, ROW_OPACITY = 0, 6, 10
LOGIT_CAP = math.log(0.01 / 0.99)


def quat_mul(a, b) -> np.ndarray:
    """Hamilton product a (x) b of (w, x, y, z) quaternions ([..., 4])."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    aw, ax, ay, az = np.moveaxis(a, -1, 0)
    bw, bx, by, bz = np.moveaxis(b, -1, 0)
    return np.stack([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw], -1)


def store_ids(params: np.ndarray, s: float) -> np.ndarray:
    return oc.encode_id(oc.chunk_coord(params[0:3].T, s))


def assign(ids: np.ndarray, s: float, keyframes: list) -> np.ndarray:
    """Index of the correction applied to each Gaussian (-1: none), given
    the EncodedID of the chunk holding it."""
    chunk_ids = np.unique(ids)
    owner = {}
    for k, (cam, _, _) in enumerate(keyframes):
        for c in oc.select_chunks([cam], chunk_ids, s)["union_ids"]:
            owner.setdefault(int(c), k)
    return np.array([owner.get(int(c), -1) for c in ids], np.int64)


def loop_closure(params, m, v, step, ids, s: float, keyframes: list, junctions: list) -> dict:
    """Apply the correction; returns the regrouped store (params, m, v,
    step as float32/int32 arrays, chunk ids), the applied correction per
    Gaussian in the new order (-1: none), and the reset mask in the new
    order."""
    P = np.array(params, np.float32, copy=True)
    old_ids = np.asarray(ids, np.uint64)
    if (old_ids[1:] < old_ids[:-1]).any():
        raise ValueError("the store must be in ascending EncodedID order")
    own = assign(old_ids, s, keyframes)
    for k, (_, R, t) in enumerate(keyframes):
        sel = own == k
        if not sel.any():
            continue
        R = np.asarray(R, np.float64)
        t = np.asarray(t, np.float64)
        x, y, z = (P[a, sel].astype(np.float64) for a in range(3))
        # elementwise, left to right, no fused operations
        mu = np.stack([((R[i, 0] * x + R[i, 1] * y) + R[i, 2] * z) + t[i] for i in range(3)])
        qr = quat_wxyz(R)
        q = quat_mul(qr[None, :], P[ROW_QUAT:ROW_QUAT + 4, sel].T.astype(np.float64)).T
        P[0:3, sel] = mu.astype(np.float32)
        P[ROW_QUAT:ROW_QUAT + 4, sel] = q.astype(np.float32)
    new_ids = np.where(own >= 0, store_ids(P, s), old_ids)
    # the store is already in the previous order: a stable sort keeps it
    order = np.argsort(new_ids, kind="stable")
    out = dict(params=P[:, order], m=np.asarray(m, np.float32)[:, order].copy(),
               v=np.asarray(v, np.float32)[:, order].copy(),
               step=np.asarray(step, np.int32)[order].copy(), owner=own[order],
               ids=new_ids[order])
    reset = np.zeros(P.shape[1], bool)
    if junctions:
        chunk_ids = np.unique(out["ids"])
        vis = set()
        for cam in junctions:
            vis |= set(int(c) for c in oc.select_chunks([cam], chunk_ids, s)["union_ids"])
        reset = np.isin(out["ids"], np.array(sorted(vis), np.uint64))
        lg = out["params"][ROW_OPACITY]
        out["params"][ROW_OPACITY] = np.where(reset, np.minimum(lg, np.float32(LOGIT_CAP)), lg)
        out["m"][:, reset] = 0.0
        out["v"][:, reset] = 0.0
        out["step"][reset] = 0
    out["reset"] = reset
    return out
