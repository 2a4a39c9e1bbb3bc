"""Oracle: chunk coordinates, chunk IDs, chunk visibility, residency, compaction.

TEST INFRASTRUCTURE ONLY (see the package header).

Functions and what pins them (tests/test_oracle_chunks.py):

* ``chunk_coord``     Sec. III-D "Chunking", Eq. (5).  Pinned by hand values
                      at cell boundaries and negative coordinates.
* ``encode_id`` / ``decode_id``   Sec. III-D, Eq. (6).  Pinned by hand values,
                      round trip over extreme coordinates, and the order
                      invariant (ascending ID == lexicographic (cx, cy, cz)).
* ``frustum_halfspaces``, ``box_visible``, ``select_chunks``
                      Sec. III-D "Frustum Culling" and Sec. III-E.  The
                      paper's hierarchical plane test is an accelerated way of
                      finding the chunks whose cubic cell meets the view
                      frustum; the oracle answers that question directly for
                      every chunk by vertex enumeration of the intersection
                      polytope.  Pinned by brute-force lattice witnesses and by
                      SciPy's LP solver (HiGHS) on small grids.
* ``residency_plan``  Sec. III-E "Optimization" and "LRU Eviction Strategy".
                      Pinned by brute force over access orders on tiny cases.
* ``compact``         Sec. III-E (index only the visible Gaussians).  Pinned by
                      permutation / count identities.
"""
from __future__ import annotations

import itertools

import numpy as np

ID_OFFSET = 1 << 20          # Eq. (6): offset added to each coordinate
ID_BITS = 21                 # Eq. (6): bits per coordinate
COORD_MIN = -(1 << 20)
COORD_MAX = (1 << 20) - 1


def chunk_coord(p, s: float) -> np.ndarray:
    """Eq. (5): floor((p_i + s/2) / s) per axis, evaluated in float64.

    `p` is [..., 3] (any float type; float32 inputs convert exactly)."""
    p = np.asarray(p, np.float64)
    return np.floor((p + s / 2.0) / s).astype(np.int64)


def encode_id(c) -> np.ndarray:
    """Eq. (6): (cx + 2^20) * 2^42 + (cy + 2^20) * 2^21 + (cz + 2^20), as uint64.

    Raises ValueError for coordinates outside [-2^20, 2^20 - 1]."""
    c = np.asarray(c, np.int64)
    if c.size and (c.min() < COORD_MIN or c.max() > COORD_MAX):
        raise ValueError("chunk coordinate outside the 21-bit range of Eq. (6)")
    sh = (c + ID_OFFSET).astype(np.uint64)
    return sh[..., 0] * np.uint64(1 << 42) + sh[..., 1] * np.uint64(1 << 21) + sh[..., 2]


def decode_id(ids) -> np.ndarray:
    ids = np.asarray(ids, np.uint64)
    mask = np.uint64((1 << ID_BITS) - 1)
    cx = (ids // np.uint64(1 << 42)) & mask
    cy = (ids // np.uint64(1 << 21)) & mask
    cz = ids & mask
    return np.stack([cx, cy, cz], axis=-1).astype(np.int64) - ID_OFFSET


# ---------------------------------------------------------------------------
# Visibility
# ---------------------------------------------------------------------------
def frustum_halfspaces(cam: dict) -> tuple[np.ndarray, np.ndarray]:
    """The view frustum F = {x : z_near <= Z <= z_far, 0 <= u <= W, 0 <= v <= H}
    as six world-space half-spaces a.x <= b with unit-length a.

    (X, Y, Z) = R x + t are camera coordinates and u = fx X/Z + cx,
    v = fy Y/Z + cy.  Since Z >= z_near > 0 inside F, each image-side
    inequality is multiplied through by Z and stays linear."""
    R, t = cam["R"], cam["t"]
    fx, fy, cx, cy = cam["fx"], cam["fy"], cam["cx"], cam["cy"]
    W, H = cam["width"], cam["height"]
    r0, r1, r2 = R
    t0, t1, t2 = t
    rows = [
        (-r2, t2 - cam["z_near"]),                                   # Z >= z_near
        (r2, cam["z_far"] - t2),                                     # Z <= z_far
        (-(fx * r0 + cx * r2), fx * t0 + cx * t2),                   # u >= 0
        (fx * r0 + (cx - W) * r2, -(fx * t0 + (cx - W) * t2)),       # u <= W
        (-(fy * r1 + cy * r2), fy * t1 + cy * t2),                   # v >= 0
        (fy * r1 + (cy - H) * r2, -(fy * t1 + (cy - H) * t2)),       # v <= H
    ]
    A = np.array([r[0] for r in rows], np.float64)
    b = np.array([r[1] for r in rows], np.float64)
    nrm = np.linalg.norm(A, axis=1)
    return A / nrm[:, None], b / nrm


_TRIPLES = np.array(list(itertools.combinations(range(12), 3)), np.int64)   # 220 triples


def _vertex_feasible(A_f, b_f, lo, hi, tol):
    """For boxes [lo, hi] (m x 3): does {x : A_f x <= b_f, lo <= x <= hi} have
    a vertex satisfying every constraint within `tol`?  A bounded non-empty
    polytope always has a vertex, and each vertex is the unique solution of
    three linearly independent active constraints, so enumerating every
    triple decides emptiness exactly (up to `tol`)."""
    m = lo.shape[0]
    eye = np.eye(3)
    A = np.concatenate([np.broadcast_to(A_f, (m, 6, 3)),
                        np.broadcast_to(-eye, (m, 3, 3)), np.broadcast_to(eye, (m, 3, 3))], axis=1)
    b = np.concatenate([np.broadcast_to(b_f, (m, 6)), -lo, hi], axis=1)
    At = A[:, _TRIPLES]                         # m x 220 x 3 x 3
    bt = b[:, _TRIPLES]                         # m x 220 x 3
    det = np.linalg.det(At)
    ok = np.abs(det) > 1e-12
    At = np.where(ok[..., None, None], At, eye)
    x = np.linalg.solve(At, bt[..., None])[..., 0]          # m x 220 x 3
    viol = np.einsum("mkj,mtj->mtk", A, x) - b[:, None, :]  # m x 220 x 12
    feas = ok & (viol.max(axis=2) <= tol)
    return feas.any(axis=1)


def box_visible(cam: dict, lo: np.ndarray, hi: np.ndarray, tie_tol: float) -> tuple[np.ndarray, np.ndarray]:
    """Closed boxes [lo, hi] (m x 3) against the closed frustum of `cam`.

    Returns (visible, tie).  `visible` uses a tolerance of 1e-3*tie_tol; `tie`
    marks boxes whose answer changes when every constraint is moved by
    +-tie_tol (metres): such boxes touch the frustum only within rounding
    distance and are excluded from bit-exact comparisons."""
    A_f, b_f = frustum_halfspaces(cam)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    vis = np.zeros(lo.shape[0], bool)
    tie = np.zeros(lo.shape[0], bool)
    for s in range(0, lo.shape[0], 512):
        sl = slice(s, s + 512)
        v0 = _vertex_feasible(A_f, b_f, lo[sl], hi[sl], 1e-3 * tie_tol)
        vp = _vertex_feasible(A_f, b_f + tie_tol, lo[sl] - tie_tol, hi[sl] + tie_tol, 1e-3 * tie_tol)
        vm = _vertex_feasible(A_f, b_f - tie_tol, lo[sl] + tie_tol, hi[sl] - tie_tol, 1e-3 * tie_tol)
        vis[sl] = v0
        tie[sl] = vp != vm
    return vis, tie


def chunk_box(coords, s: float) -> tuple[np.ndarray, np.ndarray]:
    """The closed cubic cell of chunk c under Eq. (5): [c*s - s/2, c*s + s/2]."""
    c = np.asarray(coords, np.float64)
    return c * s - s / 2.0, c * s + s / 2.0


def select_chunks(cams: list, ids: np.ndarray, s: float) -> dict:
    """For each view, the chunks (given by ascending EncodedIDs) whose cell
    meets its frustum.

    Returns ``visible`` (n_views x m bool), ``tie`` (same shape),
    ``union_ids`` (ascending uint64 ids visible in any view) and
    ``view_mask`` (uint16 per union id, bit v set when view v sees it)."""
    ids = np.asarray(ids, np.uint64)
    lo, hi = chunk_box(decode_id(ids), s)
    vis = np.zeros((len(cams), ids.size), bool)
    tie = np.zeros_like(vis)
    for v, cam in enumerate(cams):
        vis[v], tie[v] = box_visible(cam, lo, hi, 1e-9 * s)
    any_v = vis.any(axis=0)
    mask = np.zeros(ids.size, np.uint64)
    for v in range(len(cams)):
        mask |= vis[v].astype(np.uint64) << np.uint64(v)
    return dict(visible=vis, tie=tie, union_ids=ids[any_v], view_mask=mask[any_v].astype(np.uint16))


# ---------------------------------------------------------------------------
# Residency (LRU) and compaction
# ---------------------------------------------------------------------------
class BudgetError(RuntimeError):
    pass


def residency_plan(needed, resident: dict, counts: dict, budget: int, now: int) -> dict:
    """One residency decision of the mapping step.

    `needed` are the visible chunk ids, `resident` maps resident id -> last
    access time, `counts` maps id -> number of Gaussians, `budget` is the
    device budget in Gaussians.  Chunks to load are needed \\ resident.  If
    the loaded total would exceed the budget, the evictable chunks (resident
    and not needed) are taken oldest access first (ties: lower id first) and
    the shortest such prefix that makes everything fit is evicted.  If even
    evicting all of them does not fit, BudgetError.  Needed chunks get access
    time `now`.  Returns dict(load, evict, resident)."""
    needed = sorted(set(int(x) for x in needed))
    load = [c for c in needed if c not in resident]
    total = sum(counts[c] for c in resident) + sum(counts[c] for c in load)
    evictable = sorted((c for c in resident if c not in set(needed)), key=lambda c: (resident[c], c))
    evict = []
    for c in evictable:
        if total <= budget:
            break
        evict.append(c)
        total -= counts[c]
    if total > budget:
        raise BudgetError(f"visible set needs {total} Gaussians, budget {budget}")
    new_res = {c: t for c, t in resident.items() if c not in set(evict)}
    for c in needed:
        new_res[c] = now
    return dict(load=load, evict=evict, resident=new_res)


def compact(active_ids, chunk_arrays: dict) -> tuple[np.ndarray, np.ndarray]:
    """Concatenate the active chunks' Gaussians in ascending id order.

    `chunk_arrays` maps id -> (params [R, n_c], slot_ids [n_c]).  Returns the
    compacted params and the slot id of every compacted Gaussian."""
    ids = sorted(int(x) for x in active_ids)
    ps = [chunk_arrays[c][0] for c in ids]
    ss = [chunk_arrays[c][1] for c in ids]
    if not ps:
        return np.zeros((0, 0), np.float32), np.zeros(0, np.int64)
    return np.concatenate(ps, axis=1), np.concatenate(ss)
