"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This module draws random numbers and lays them out; it holds none of the
method's arithmetic (no projection, no chunking, no compositing).  Every
generator takes an explicit seed and uses NumPy's PCG64, so the same call
gives the same arrays on every machine.

Parameter block layout (the interface both sides read; see ``include/dcgs.h``):
one float32 array ``params[R, n]`` with R = 11 + 3*K, K = (deg+1)^2 rows

    0..2    mean x, y, z (world, metres)
    3..5    log-scale along the three local axes
    6..9    quaternion w, x, y, z (not normalised)
    10      opacity logit
    11+3k+c SH coefficient k (k = l*l + l + m) of colour channel c

Cameras are dicts of float64 values: ``R`` (3x3, world->camera rotation),
``t`` (3, world->camera translation), ``fx, fy, cx, cy``, ``width``,
``height``, ``z_near``, ``z_far``.  Camera axes: x right, y down, z forward.

The workloads follow the shapes of the paper's indoor and driving
experiments (synthetic stand-ins for the datasets the paper evaluates on).
"""
from __future__ import annotations

import math

import numpy as np

ROW_MEAN = 0
ROW_LOG_SCALE = 3
ROW_QUAT = 6
ROW_OPACITY = 10
ROW_SH = 11

# The degree-0 coefficient that makes a Gaussian's colour exactly `rgb`
# is (rgb - 0.5) * 2*sqrt(pi): a distribution parameter of the generator.
_DC_FROM_RGB = 2.0 * math.sqrt(math.pi)


def n_rows(sh_degree: int) -> int:
    return 11 + 3 * (sh_degree + 1) ** 2


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _fill_common(rng, params, n, log_scale_mu, log_scale_sd, sh_degree, rest_sd):
    params[ROW_LOG_SCALE:ROW_LOG_SCALE + 3] = rng.normal(log_scale_mu, log_scale_sd, (3, n))
    q = rng.normal(0.0, 1.0, (4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    params[ROW_QUAT:ROW_QUAT + 4] = q
    params[ROW_OPACITY] = rng.normal(0.0, 1.0, n)
    rgb = rng.uniform(0.0, 1.0, (3, n))
    params[ROW_SH:ROW_SH + 3] = (rgb - 0.5) * _DC_FROM_RGB
    k = (sh_degree + 1) ** 2
    if k > 1:
        params[ROW_SH + 3:ROW_SH + 3 * k] = rng.normal(0.0, rest_sd, (3 * (k - 1), n))


def camera(R, t, fx, fy, cx, cy, width, height, z_near=0.2, z_far=1000.0) -> dict:
    return dict(R=np.asarray(R, np.float64).reshape(3, 3), t=np.asarray(t, np.float64).reshape(3),
                fx=float(fx), fy=float(fy), cx=float(cx), cy=float(cy),
                width=int(width), height=int(height), z_near=float(z_near), z_far=float(z_far))


def look_camera(position, yaw, pitch, fx, fy, width, height, z_near=0.2, z_far=1000.0, cx=None, cy=None):
    """Camera at `position` (world, z up) looking along yaw/pitch (radians)."""
    f = np.array([math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw), math.sin(pitch)])
    right = np.cross(f, [0.0, 0.0, 1.0])
    right /= np.linalg.norm(right)
    down = np.cross(f, right)
    R_wc = np.stack([right, down, f], axis=1)
    R = R_wc.T
    t = -R @ np.asarray(position, np.float64)
    return camera(R, t, fx, fy, width / 2.0 if cx is None else cx, height / 2.0 if cy is None else cy,
                  width, height, z_near, z_far)


# --------------------------------------------------------------------------
# Tiny scene: one view, one chunk, SH degree 0.
# --------------------------------------------------------------------------
def tiny_scene(n: int = 10_000, seed: int = 0, width: int = 256, height: int = 192,
               focal: float = 200.0, sh_degree: int = 0, rest_sd: float = 0.05) -> dict:
    """Means uniform in [-2,2]^2 x [2,6] in front of an identity-pose camera;
    log-scales N(-3.5, 0.5); uniform unit quaternions; logits N(0,1);
    colour U(0,1) through the degree-0 coefficient (higher SH N(0, rest_sd^2)
    when sh_degree > 0)."""
    rng = _rng(seed)
    params = np.zeros((n_rows(sh_degree), n), np.float64)
    params[0] = rng.uniform(-2.0, 2.0, n)
    params[1] = rng.uniform(-2.0, 2.0, n)
    params[2] = rng.uniform(2.0, 6.0, n)
    _fill_common(rng, params, n, -3.5, 0.5, sh_degree, rest_sd)
    cam = camera(np.eye(3), np.zeros(3), focal, focal, width / 2.0, height / 2.0, width, height)
    return dict(params=params.astype(np.float32), sh_degree=sh_degree, camera=cam, chunk_size=16.0)


def target_image(width: int, height: int, seed: int = 1, channels: int = 3) -> np.ndarray:
    """Seeded U(0,1) target image, planar [channels, H, W] float32."""
    return _rng(seed).uniform(0.0, 1.0, (channels, height, width)).astype(np.float32)


def upstream_grad(width: int, height: int, seed: int, channels: int = 3, scale: float = 1.0) -> np.ndarray:
    """Seeded N(0, scale^2) array shaped like an image: an upstream gradient."""
    return (_rng(seed).normal(0.0, 1.0, (channels, height, width)) * scale).astype(np.float32)


# --------------------------------------------------------------------------
# Indoor room: floor and four walls of an 8 x 8 x 3 m room.
# --------------------------------------------------------------------------
ROOM = (8.0, 8.0, 3.0)


def room_scene(n: int, seed: int = 10, sh_degree: int = 3, jitter: float = 0.02,
               log_scale_mu: float = -3.5, log_scale_sd: float = 0.5, rest_sd: float = 0.05) -> dict:
    """Gaussians on the floor (z=0) and four walls, allocated by area, with
    N(0, jitter^2) offsets off the planes."""
    rng = _rng(seed)
    Lx, Ly, Lz = ROOM
    areas = np.array([Lx * Ly, Ly * Lz, Ly * Lz, Lx * Lz, Lx * Lz])
    counts = np.floor(n * areas / areas.sum()).astype(np.int64)
    counts[0] += n - counts.sum()
    pts = []
    for plane, c in enumerate(counts):
        a = rng.uniform(0.0, 1.0, c)
        b = rng.uniform(0.0, 1.0, c)
        p = np.zeros((3, c))
        if plane == 0:
            p[0], p[1], p[2] = a * Lx, b * Ly, 0.0
        elif plane in (1, 2):
            p[0], p[1], p[2] = (0.0 if plane == 1 else Lx), a * Ly, b * Lz
        else:
            p[0], p[1], p[2] = a * Lx, (0.0 if plane == 3 else Ly), b * Lz
        pts.append(p)
    mean = np.concatenate(pts, axis=1) + rng.normal(0.0, jitter, (3, n))
    params = np.zeros((n_rows(sh_degree), n), np.float64)
    params[0:3] = mean
    _fill_common(rng, params, n, log_scale_mu, log_scale_sd, sh_degree, rest_sd)
    return dict(params=params.astype(np.float32), sh_degree=sh_degree)


def perturb(params: np.ndarray, seed: int = 12, dc_sd: float = 0.1, logit_sd: float = 0.5,
            mean_sd: float = 0.01) -> np.ndarray:
    """A perturbed copy of a scene, the starting point of optimisation."""
    rng = _rng(seed)
    out = params.copy()
    n = out.shape[1]
    # sums in float64, rounded once to float32; only the touched rows widen
    out[0:3] = (params[0:3].astype(np.float64) + rng.normal(0.0, mean_sd, (3, n))).astype(np.float32)
    out[ROW_OPACITY] = (params[ROW_OPACITY].astype(np.float64)
                        + rng.normal(0.0, logit_sd, n)).astype(np.float32)
    out[ROW_SH:ROW_SH + 3] = (params[ROW_SH:ROW_SH + 3].astype(np.float64)
                              + rng.normal(0.0, dc_sd, (3, n))).astype(np.float32)
    return out


def room_trajectory(n_frames: int, seed: int = 11, width: int = 1200, height: int = 680,
                    focal: float = 600.0, z_far: float = 6.0, z_near: float = 0.2,
                    max_step: float = 0.05) -> list:
    """Smooth random walk: AR(1)-smoothed velocity capped at `max_step` m per
    frame, x, y in [1, 7], z in [1.2, 1.8], smooth yaw, pitch within +-10 deg."""
    rng = _rng(seed)
    pos = np.array([4.0, 4.0, 1.5])
    vel = np.zeros(3)
    yaw = rng.uniform(-math.pi, math.pi)
    yaw_rate = 0.0
    cams = []
    for _ in range(n_frames):
        vel = 0.9 * vel + 0.1 * rng.normal(0.0, max_step, 3) * np.array([1.0, 1.0, 0.3])
        sp = np.linalg.norm(vel)
        if sp > max_step:
            vel *= max_step / sp
        pos = pos + vel
        for ax, lo, hi in ((0, 1.0, 7.0), (1, 1.0, 7.0), (2, 1.2, 1.8)):
            if pos[ax] < lo or pos[ax] > hi:
                pos[ax] = min(max(pos[ax], lo), hi)
                vel[ax] = -vel[ax]
        yaw_rate = 0.95 * yaw_rate + 0.05 * rng.normal(0.0, 0.05)
        yaw += yaw_rate
        pitch = math.radians(10.0) * math.sin(0.01 * len(cams) + seed)
        cams.append(look_camera(pos.copy(), yaw, pitch, focal, focal, width, height, z_near, z_far))
    return cams


# --------------------------------------------------------------------------
# Small chunk grids for visibility tests.
# --------------------------------------------------------------------------
def random_cameras(n: int, seed: int, extent: float, width: int = 64, height: int = 48,
                   focal: float = 40.0, z_near: float = 0.2, z_far: float = 3.0) -> list:
    """Cameras at random positions in [-extent, extent]^3 with random
    orientation (SciPy's uniform random rotation)."""
    from scipy.spatial.transform import Rotation

    rng = _rng(seed)
    cams = []
    for _ in range(n):
        R = Rotation.random(random_state=rng).as_matrix()
        C = rng.uniform(-extent, extent, 3)
        cams.append(camera(R, -R @ C, focal * rng.uniform(0.5, 2.0), focal * rng.uniform(0.5, 2.0),
                           width / 2.0, height / 2.0, width, height, z_near,
                           z_far * rng.uniform(0.5, 2.0)))
    return cams


def grid_coords(n_side: int, offset: int = -3) -> np.ndarray:
    """All integer chunk coordinates of an n_side^3 block, int64 [m, 3]."""
    r = np.arange(n_side) + offset
    cx, cy, cz = np.meshgrid(r, r, r, indexing="ij")
    return np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1).astype(np.int64)


def adam_inputs(n_rows_: int, n: int, seed: int, n_slots: int | None = None) -> dict:
    """Random parameters, gradients, moments and step counters for optimiser
    tests; `src` is a random injective map from n compacted entries into
    n_slots pool slots."""
    rng = _rng(seed)
    n_slots = n if n_slots is None else n_slots
    src = rng.permutation(n_slots)[:n].astype(np.int32)
    return dict(
        params=rng.normal(0.0, 1.0, (n_rows_, n_slots)).astype(np.float32),
        m=rng.normal(0.0, 1e-3, (n_rows_, n_slots)).astype(np.float32),
        v=np.abs(rng.normal(0.0, 1e-6, (n_rows_, n_slots))).astype(np.float32),
        step=rng.integers(0, 50, n_slots).astype(np.int32),
        grad=(rng.normal(0.0, 1e-4, (n_rows_, n)) * (rng.uniform(0, 1, (n_rows_, n)) > 0.1)).astype(np.float32),
        src=src)


# --------------------------------------------------------------------------
# Driving corridor: road and facades along a piecewise-straight path.
# --------------------------------------------------------------------------
CELL = 50.0          # grid cell of the corridor layout (m)
GRID = 64            # cells per side
ROAD_HALF = 15.0     # half width of the road (m)
FACADE_H = 10.0      # facade height (m)
PATH_OFFSET = 0.3    # centre-line offset from the layout cell centres (m)


def driving_path(seed: int = 20, length: float = 4000.0, max_tries: int = 200) -> np.ndarray:
    """Centre line of a corridor: straight segments of 200-600 m (multiples of
    50 m) joined by +-90 degree turns, inside a 64 x 64 grid of 50 m cells,
    never re-entering a cell it already crossed.  Returns [m, 2] points 1 m
    apart."""
    for attempt in range(max_tries):
        rng = _rng(seed * 1000 + attempt)
        cx, cy = 4, 4
        dirs = [(1, 0), (0, 1), (-1, 0), (0, -1)]
        d = int(rng.integers(0, 2))
        used = {(cx, cy)}
        cells = [(cx, cy)]
        total = 0.0
        ok = True
        while total < length:
            seg = int(rng.integers(4, 13))          # 200..600 m
            dx, dy = dirs[d]
            path = [(cx + dx * k, cy + dy * k) for k in range(1, seg + 1)]
            if any(not (3 <= x < GRID - 3 and 3 <= y < GRID - 3) or (x, y) in used
                   or any((x + ex, y + ey) in used and (x + ex, y + ey) != (cx, cy)
                          and (x + ex, y + ey) not in path
                          for ex, ey in ((1, 0), (-1, 0), (0, 1), (0, -1)))
                   for x, y in path):
                ok = False
                break
            used.update(path)
            cells.extend(path)
            cx, cy = path[-1]
            total += seg * CELL
            d = (d + (1 if rng.uniform() < 0.5 else 3)) % 4
        if ok:
            # centre line 0.3 m off the cell centres, so that no camera
            # position lies on a chunk face of Eq. (5)
            pts = np.array(cells, np.float64) * CELL + CELL / 2 + PATH_OFFSET
            out = [pts[0]]
            for a, b in zip(pts[:-1], pts[1:]):
                n = int(round(np.linalg.norm(b - a)))
                for k in range(1, n + 1):
                    out.append(a + (b - a) * k / n)
            return np.array(out)[: int(length) + 1]
    raise RuntimeError("no corridor layout found")


def driving_scene(n: int, seed: int = 20, sh_degree: int = 3, path: np.ndarray | None = None,
                  jitter: float = 0.02, log_scale_mu: float = -2.5, log_scale_sd: float = 0.5,
                  rest_sd: float = 0.05, chunked: int = 1 << 22) -> dict:
    """Gaussians on the road (z = 0, 30 m wide) and two facades (+-15 m,
    z in [0, 10]) along the corridor, allocated by area, N(0, jitter^2)
    offsets; SH degree 3 colours as in the indoor scene.  Generated in
    blocks to bound memory."""
    P = driving_path(seed) if path is None else path
    rng = _rng(seed + 7)
    seg_len = np.linalg.norm(np.diff(P, axis=0), axis=1)
    L = seg_len.sum()
    road, facade = 2 * ROAD_HALF * L, 2 * FACADE_H * L
    n_road = int(round(n * road / (road + facade)))
    params = np.zeros((n_rows(sh_degree), n), np.float32)
    cum = np.concatenate([[0.0], np.cumsum(seg_len)])
    for s0 in range(0, n, chunked):
        m = min(chunked, n - s0)
        idx = np.arange(s0, s0 + m)
        t = rng.uniform(0.0, L, m)
        k = np.clip(np.searchsorted(cum, t, "right") - 1, 0, len(seg_len) - 1)
        f = (t - cum[k]) / np.maximum(seg_len[k], 1e-9)
        base = P[k] + (P[k + 1] - P[k]) * f[:, None]
        tang = (P[k + 1] - P[k]) / np.maximum(seg_len[k], 1e-9)[:, None]
        nrm = np.stack([-tang[:, 1], tang[:, 0]], 1)
        is_road = idx < n_road
        lateral = np.where(is_road, rng.uniform(-ROAD_HALF, ROAD_HALF, m),
                           np.where(rng.uniform(0, 1, m) < 0.5, -ROAD_HALF, ROAD_HALF))
        z = np.where(is_road, 0.0, rng.uniform(0.0, FACADE_H, m))
        xy = base + nrm * lateral[:, None]
        block = np.zeros((n_rows(sh_degree), m), np.float64)
        block[0], block[1], block[2] = xy[:, 0], xy[:, 1], z
        block[0:3] += rng.normal(0.0, jitter, (3, m))
        _fill_common(rng, block, m, log_scale_mu, log_scale_sd, sh_degree, rest_sd)
        params[:, s0:s0 + m] = block
    return dict(params=params, sh_degree=sh_degree, path=P)


def driving_trajectory(path: np.ndarray, n_frames: int | None = None, width: int = 1241,
                       height: int = 376, focal: float = 718.0, z_far: float = 350.0,
                       z_near: float = 0.2, cam_height: float = 1.65, start: int = 0,
                       turn_frames: int = 15) -> list:
    """Forward-facing camera on the centre line at 1 m per frame; the yaw is
    eased over +-turn_frames around each corner."""
    m = len(path) if n_frames is None else min(len(path), start + n_frames)
    d = np.diff(path, axis=0)
    yaw = np.unwrap(np.arctan2(d[:, 1], d[:, 0]))
    yaw = np.concatenate([yaw, yaw[-1:]])
    kern = np.ones(2 * turn_frames + 1) / (2 * turn_frames + 1)
    pad = np.pad(yaw, turn_frames, mode="edge")
    yaw_s = np.convolve(pad, kern, mode="valid")
    cams = []
    for k in range(start, m):
        pos = np.array([path[k, 0], path[k, 1], cam_height])
        cams.append(look_camera(pos, float(yaw_s[k]), 0.0, focal, focal, width, height, z_near,
                                z_far, cx=width / 2.0, cy=height / 2.0))
    return cams


def mlp_init(seed: int, in_dim: int = 59, hidden: int = 256, bias_sd: float = 0.0) -> np.ndarray:
    """Initial flat float32 parameters of the prefetch network (layout W1
    [hidden][in], b1, W2 [hidden][hidden], b2, w3 [hidden], b3): weights
    U(-1/sqrt(fan_in), 1/sqrt(fan_in)), biases N(0, bias_sd^2)."""
    rng = _rng(seed)
    parts = []
    for fan_in, n_out in ((in_dim, hidden), (hidden, hidden), (hidden, 1)):
        a = 1.0 / math.sqrt(fan_in)
        parts.append(rng.uniform(-a, a, fan_in * n_out))
        parts.append(rng.normal(0.0, 1.0, n_out) * bias_sd)
    return np.concatenate(parts).astype(np.float32)
