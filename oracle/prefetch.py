"""Oracle: learned chunk prefetch -- candidate cells, pose features, exact
visibility labels, and the prefetch MLP (forward, loss, gradients, Adam),
all in float64.

TEST INFRASTRUCTURE ONLY (see the package header).

The paper streams chunks in and out by the exact frustum test of each frame
(Sec. III-D "Frustum Culling", Sec. III-E "Optimization"), and points to
pose-aware caching as what keeps that cheap.  The prefetcher built on top
predicts, from the recent camera poses, which chunk cells the exact test
will select in the next few frames, so that their host-to-device staging
can start before they are needed.  The paper does not define it; the
definitions below are this implementation's, and the exact test stays the
judge (a cell it selects that was not staged is loaded on demand).

Definitions (all vectors expressed in the frame of the current camera,
R0 = its world-to-camera rotation, c0 = its centre):

* history: frames t, t-1, ..., t-7 (earlier indices clamp to 0);
* pose feature of history entry k: R0 (c_k - c0) / pos_unit (3 values) and
  the unit quaternion (w, x, y, z), w >= 0, of R0 R_k^T (4 values);
  56 values for the 8 entries, entry 0 first;
* candidates: the 64 x 64 x 1 chunk cells (Eq. 5) around the cell holding
  c0, cell (bx + i - 32, by + j - 32, bz + k) for candidate q = (k*64 + j)*64
  + i; the offset feature of a cell is R0 (cell_centre - c0) / (8 s);
* input row of a candidate: the 56 pose values, then its 3 offset values;
* label of a candidate at frame t: 1 when its closed cell meets the frustum
  of any of frames t+1 .. t+horizon (those that exist), else 0;
* network: z1 = W1 x + b1, h1 = GELU(z1), z2 = W2 h1 + b2, h2 = GELU(z2),
  logit = w3 . h2 + b3, P(visible) = sigmoid(logit); GELU is the exact
  z * Phi(z); weights W1, W2, w3 are used rounded to bfloat16 (round to
  nearest even) from float32 master values, biases in float32;
* loss: mean over the batch of wp * y * softplus(-logit) + (1 - y) *
  softplus(logit) (binary cross-entropy with a positive-class weight wp);
* optimiser: Adam on the float32 master vector with bias correction; the
  bfloat16 copy is re-rounded after each step.

Flat parameter vector (float32 master, 81,409 values for 59 -> 256 -> 256
-> 1): W1 [256][59] row-major, b1 [256], W2 [256][256], b2 [256], w3 [256],
b3 [1].  The bfloat16 copy holds W1, W2, w3 back to back.

What pins each function (tests/test_oracle_prefetch.py):

* ``quat_wxyz``       rotation matrix rebuilt from the quaternion by the
                      textbook formula; yaw rotations in closed form.
* ``pose_features``   straight-line and constant-yaw-rate trajectories in
                      closed form.
* ``candidate_cells`` / ``cell_offsets``  hand-placed cells ahead of, left
                      of and behind the camera.
* ``labels``          dense sampling of the future frusta: every cell that
                      holds a sample point is labelled visible.
* ``bf16_round``      torch's float32 -> bfloat16 conversion.
* ``gelu``            scipy.stats.norm.cdf, special values.
* ``mlp_forward`` / ``bce``   torch.nn.functional layers in float64.
* ``mlp_grad``        central finite differences on a small network.
* ``adam``            the first step from zero moments in closed form.
"""
from __future__ import annotations

import math

import numpy as np
import torch
from scipy.spatial.transform import Rotation

from . import chunks as oc

HIST = 8
GRID = (64, 64, 1)
OFFSET_UNIT = 8.0       # cell offsets in units of 8 chunk sides
IN_DIM = HIST * 7 + 3   # 59
HIDDEN = 256


def layout(in_dim: int = IN_DIM, hidden: int = HIDDEN) -> dict:
    """Offsets of the flat master vector and of the bfloat16 weight copy."""
    o, off = 0, {}
    for name, size in (("W1", hidden * in_dim), ("b1", hidden), ("W2", hidden * hidden),
                       ("b2", hidden), ("w3", hidden), ("b3", 1)):
        off[name] = (o, size)
        o += size
    off["total"] = o
    ob, offb = 0, {}
    for name in ("W1", "W2", "w3"):
        offb[name] = (ob, off[name][1])
        ob += off[name][1]
    offb["total"] = ob
    return dict(master=off, bf16=offb, in_dim=in_dim, hidden=hidden)


# ---------------------------------------------------------------------------
# Features
# ---------------------------------------------------------------------------
def centre(cam: dict) -> np.ndarray:
    """Camera centre in world coordinates: -R^T t."""
    return -cam["R"].T @ cam["t"]


def quat_wxyz(Rm: np.ndarray) -> np.ndarray:
    """Unit quaternion (w, x, y, z) of a rotation matrix, w >= 0."""
    x, y, z, w = Rotation.from_matrix(np.asarray(Rm, np.float64)).as_quat()
    q = np.array([w, x, y, z])
    return -q if q[0] < 0 else q


def history(cams: list, t: int) -> list:
    """Cameras of frames t, t-1, ..., t-7 (indices below 0 clamp to 0)."""
    return [cams[max(t - k, 0)] for k in range(HIST)]


def pose_features(hist: list, pos_unit: float = 1.0) -> np.ndarray:
    R0, c0 = hist[0]["R"], centre(hist[0])
    out = []
    for cam in hist:
        out.extend(R0 @ (centre(cam) - c0) / pos_unit)
        out.extend(quat_wxyz(R0 @ cam["R"].T))
    return np.array(out)


def candidate_cells(cam: dict, s: float, grid=GRID) -> np.ndarray:
    """[4096, 3] int64 cell coordinates, candidate q = (k*gy + j)*gx + i."""
    gx, gy, gz = grid
    b = oc.chunk_coord(centre(cam), s)
    k, j, i = np.meshgrid(np.arange(gz), np.arange(gy), np.arange(gx), indexing="ij")
    return np.stack([b[0] + i.ravel() - gx // 2, b[1] + j.ravel() - gy // 2,
                     b[2] + k.ravel() - gz // 2], 1).astype(np.int64)


def cell_offsets(cam: dict, cells: np.ndarray, s: float) -> np.ndarray:
    c0 = centre(cam)
    return (cam["R"] @ (cells * s - c0).T).T / (OFFSET_UNIT * s)


def features(cams: list, t: int, s: float, pos_unit: float = 1.0, grid=GRID) -> tuple:
    """Input rows [4096, 59] of frame t and the candidates' EncodedIDs."""
    hist = history(cams, t)
    cells = candidate_cells(cams[t], s, grid)
    pf = pose_features(hist, pos_unit)
    X = np.concatenate([np.broadcast_to(pf, (cells.shape[0], pf.size)),
                        cell_offsets(cams[t], cells, s)], 1)
    return X, oc.encode_id(cells)


def labels(cams: list, t: int, s: float, horizon: int = 5, grid=GRID) -> tuple:
    """Exact labels of frame t's candidates and their tie flags."""
    cells = candidate_cells(cams[t], s, grid)
    lo, hi = oc.chunk_box(cells, s)
    vis = np.zeros(cells.shape[0], bool)
    sure = np.zeros(cells.shape[0], bool)   # visible in a view without a tie
    tie = np.zeros(cells.shape[0], bool)
    for h in range(1, horizon + 1):
        if t + h >= len(cams):
            break
        v, ti = oc.box_visible(cams[t + h], lo, hi, 1e-9 * s)
        vis |= v
        sure |= v & ~ti
        tie |= ti
    return vis.astype(np.uint8), tie & ~sure


# ---------------------------------------------------------------------------
# Network
# ---------------------------------------------------------------------------
def bf16_round(x) -> np.ndarray:
    """float32 -> nearest bfloat16 (ties to even), returned as float32."""
    u = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    r = (u + np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))) & np.uint64(0xFFFF0000)
    return r.astype(np.uint32).view(np.float32)


def gelu(z):
    """Exact GELU z * Phi(z) (torch float64 tensor in, out)."""
    return 0.5 * z * (1.0 + torch.erf(z / math.sqrt(2.0)))


def unpack(theta: np.ndarray, lay: dict) -> dict:
    """Float64 tensors of the weights as the forward uses them: W1, W2, w3
    rounded to bfloat16 from the float32 master, biases as stored."""
    m = lay["master"]
    th = np.asarray(theta, np.float32)
    out = {}
    for name in ("W1", "b1", "W2", "b2", "w3", "b3"):
        o, n = m[name]
        v = th[o:o + n]
        if name in ("W1", "W2", "w3"):
            v = bf16_round(v)
        out[name] = torch.tensor(v.astype(np.float64))
    h, d = lay["hidden"], lay["in_dim"]
    out["W1"] = out["W1"].reshape(h, d)
    out["W2"] = out["W2"].reshape(h, h)
    return out


def mlp_forward(w: dict, X) -> dict:
    X = torch.as_tensor(np.asarray(X, np.float64)) if not torch.is_tensor(X) else X
    z1 = X @ w["W1"].T + w["b1"]
    h1 = gelu(z1)
    z2 = h1 @ w["W2"].T + w["b2"]
    h2 = gelu(z2)
    logit = h2 @ w["w3"] + w["b3"][0]
    return dict(z1=z1, h1=h1, z2=z2, h2=h2, logit=logit)


def sigmoid(x):
    return 1.0 / (1.0 + torch.exp(-x))


def softplus(x):
    return torch.where(x > 0, x + torch.log1p(torch.exp(-x)), torch.log1p(torch.exp(x)))


def bce(logit, y, pos_weight: float = 1.0):
    y = torch.as_tensor(np.asarray(y, np.float64))
    return torch.mean(pos_weight * y * softplus(-logit) + (1.0 - y) * softplus(logit))


def mlp_grad(theta: np.ndarray, X, y, pos_weight: float, lay: dict) -> tuple:
    """Loss and its gradient with respect to the flat parameters (the
    weights' gradient is taken at their bfloat16 values)."""
    w = unpack(theta, lay)
    for v in w.values():
        v.requires_grad_(True)
    f = mlp_forward(w, X)
    loss = bce(f["logit"], y, pos_weight)
    loss.backward()
    g = np.zeros(lay["master"]["total"])
    for name in ("W1", "b1", "W2", "b2", "w3", "b3"):
        o, n = lay["master"][name]
        g[o:o + n] = w[name].grad.reshape(-1).numpy()
    return float(loss.detach()), g


def adam(theta, m, v, g, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (step = 1 for the first); float64 arithmetic on the
    given values.  Returns theta, m, v."""
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return np.asarray(theta, np.float64) - lr * mh / (np.sqrt(vh) + eps), m, v
