"""Pins of the prefetch oracle (features, labels, network) against closed
forms, library routines, dense sampling and finite differences."""
import math

import numpy as np
import pytest
import scipy.stats
import torch
from scipy.spatial.transform import Rotation

import scenegen
from oracle import chunks as oc
from oracle import prefetch as op


def _rot_from_quat(q):
    """Textbook rotation matrix of a unit quaternion (w, x, y, z)."""
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def test_quaternion_rebuilds_rotation():
    Rs = Rotation.random(50, random_state=3).as_matrix()
    for Rm in Rs:
        q = op.quat_wxyz(Rm)
        assert q[0] >= 0 and abs(np.linalg.norm(q) - 1) < 1e-12
        assert np.abs(_rot_from_quat(q) - Rm).max() < 1e-12
    assert np.allclose(op.quat_wxyz(np.eye(3)), [1, 0, 0, 0])


def _line(n, yaw_rate=0.0, speed=1.0):
    cams, yaw, pos = [], 0.3, np.array([10.0, 20.0, 1.65])
    for k in range(n):
        cams.append(scenegen.look_camera(pos.copy(), yaw, 0.0, 500, 500, 640, 480, 0.2, 100.0))
        pos += speed * np.array([math.cos(yaw), math.sin(yaw), 0.0])
        yaw += yaw_rate
    return cams


def test_pose_features_straight_line():
    cams = _line(12, speed=1.5)
    pf = op.pose_features(op.history(cams, 10), pos_unit=0.5).reshape(8, 7)
    for k in range(8):
        # camera k frames back sits 1.5 k m behind along the optical axis (+z)
        assert np.allclose(pf[k, :3], [0.0, 0.0, -1.5 * k / 0.5], atol=1e-12)
        assert np.allclose(pf[k, 3:], [1, 0, 0, 0], atol=1e-12)
    # clamping at the start: frame 2's history repeats frame 0
    pf2 = op.pose_features(op.history(cams, 2)).reshape(8, 7)
    assert np.allclose(pf2[2], pf2[3]) and np.allclose(pf2[7], pf2[2])


def test_pose_features_constant_yaw_rate():
    w = 0.05
    cams = _line(12, yaw_rate=w, speed=0.0)
    pf = op.pose_features(op.history(cams, 9)).reshape(8, 7)
    for k in range(8):
        assert np.allclose(pf[k, :3], 0.0, atol=1e-12)
        # k frames back the heading was k w smaller (clockwise seen from
        # above), so that camera's optical axis points to the current
        # camera's right: (sin kw, 0, cos kw) in the current frame, the
        # image of (0, 0, 1) under a rotation by +kw about the camera y axis
        ang = k * w
        expect = np.array([math.cos(ang / 2), 0.0, math.sin(ang / 2), 0.0])
        R_rel = _rot_from_quat(pf[k, 3:])
        assert np.allclose(R_rel @ [0, 0, 1], [math.sin(ang), 0, math.cos(ang)], atol=1e-12)
        assert np.allclose(pf[k, 3:], expect, atol=1e-12), (k, pf[k, 3:])


def test_candidate_cells_and_offsets():
    s = 50.0
    cam = scenegen.look_camera(np.array([60.0, -40.0, 1.65]), 0.0, 0.0, 500, 500, 640, 480)
    cells = op.candidate_cells(cam, s)
    assert cells.shape == (4096, 3)
    b = oc.chunk_coord(op.centre(cam), s)
    assert (b == [1, -1, 0]).all()
    q = lambda i, j: j * 64 + i  # noqa: E731
    assert (cells[q(32, 32)] == b).all()
    assert (cells[q(0, 0)] == b + [-32, -32, 0]).all()
    assert (cells[q(63, 63)] == b + [31, 31, 0]).all()
    off = op.cell_offsets(cam, cells, s)
    # camera looks along +x: right = -y world, down = -z world, forward = +x
    c0 = np.array([60.0, -40.0, 1.65])
    ahead = cells[q(35, 32)]                     # 3 cells along +x
    d = ahead * s - c0
    assert np.allclose(off[q(35, 32)], [-d[1], -d[2], d[0]] / np.float64(8 * s), atol=1e-12)
    left = cells[q(32, 34)]                      # +y world is the camera's left (-x)
    d = left * s - c0
    assert np.allclose(off[q(32, 34)], [-d[1], -d[2], d[0]] / np.float64(8 * s), atol=1e-12)
    assert off[q(32, 34)][0] < 0 and off[q(29, 32)][2] < 0
    X, ids = op.features(_line(3), 2, s)
    assert X.shape == (4096, 59) and ids.dtype == np.uint64
    assert (np.diff(X[:, :56], axis=0) == 0).all()


def test_labels_cover_sampled_frustum_points():
    s = 50.0
    path = scenegen.driving_path(101, length=600.0)
    cams = scenegen.driving_trajectory(path, 40, width=320, height=100, focal=180.0, z_far=220.0)
    t, horizon = 20, 5
    lab, tie = op.labels(cams, t, s, horizon)
    cells = op.candidate_cells(cams[t], s)
    index = {tuple(c): k for k, c in enumerate(cells)}
    hit = np.zeros(4096, bool)
    rng = np.random.default_rng(4)
    for h in range(1, horizon + 1):
        cam = cams[t + h]
        u = rng.uniform(0, cam["width"], 20000)
        v = rng.uniform(0, cam["height"], 20000)
        z = cam["z_near"] + (cam["z_far"] - cam["z_near"]) * rng.uniform(0, 1, 20000) ** 0.5
        Xc = np.stack([(u - cam["cx"]) * z / cam["fx"], (v - cam["cy"]) * z / cam["fy"], z], 1)
        Pw = (cam["R"].T @ (Xc - cam["t"]).T).T
        for c in oc.chunk_coord(Pw, s):
            if c[2] != cells[0, 2]:
                continue                # other layers are not candidates
            k = index.get(tuple(c))
            assert k is not None        # the 64 x 64 window covers the frusta
            hit[k] = True
    assert (lab[hit] == 1).all()
    assert hit.sum() >= 5 and lab.sum() <= 3 * hit.sum() + 20
    # the last frame has no future frames
    lab_end, _ = op.labels(cams, len(cams) - 1, s, horizon)
    assert lab_end.sum() == 0


def test_labels_use_exactly_the_next_horizon_frames():
    s = 50.0
    pos = np.array([1000.0, 1000.0, 1.65])
    yaws = [math.pi / 2] + [0.0] * 4 + [math.pi] + [0.0] * 3
    cams = [scenegen.look_camera(pos, y, 0.0, 300, 300, 320, 240, 0.2, 200.0) for y in yaws]
    cells = op.candidate_cells(cams[0], s)
    q = lambda i, j: j * 64 + i  # noqa: E731
    lab5, _ = op.labels(cams, 0, s, horizon=5)
    lab4, _ = op.labels(cams, 0, s, horizon=4)
    # 3 cells behind (-x) are seen only by frame 5; 3 cells along +y only by
    # frame 0 itself, which is not part of its own label
    assert lab5[q(29, 32)] == 1 and lab4[q(29, 32)] == 0
    assert lab5[q(32, 35)] == 0
    assert lab5[q(35, 32)] == 1 and lab4[q(35, 32)] == 1
    assert (cells[q(29, 32)] == oc.chunk_coord(pos, s) + [-3, 0, 0]).all()


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=5000).astype(np.float32),
                        rng.normal(size=1000).astype(np.float32) * 1e-30,
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38], np.float32)])
    # exact ties: 1 + 2^-8 (rounds to even 1.0) and 1 + 3*2^-8 (rounds up)
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert (op.bf16_round(x).view(np.uint32) == ref.view(np.uint32)).all()
    assert op.bf16_round(np.float32(1.00390625)) == 1.0
    assert op.bf16_round(np.float32(1.01171875)) == np.float32(1.015625)


def test_gelu_special_values_and_normal_cdf():
    z = np.linspace(-8, 8, 101)
    g = op.gelu(torch.tensor(z)).numpy()
    assert np.allclose(g, z * scipy.stats.norm.cdf(z), atol=1e-15, rtol=1e-13)
    assert op.gelu(torch.tensor(0.0)).item() == 0.0
    assert abs(op.gelu(torch.tensor(40.0)).item() - 40.0) < 1e-12
    assert abs(op.gelu(torch.tensor(-40.0)).item()) < 1e-12


def _small_layout():
    return op.layout(in_dim=5, hidden=7)


def _theta(lay, seed):
    return scenegen.mlp_init(seed, lay["in_dim"], lay["hidden"], bias_sd=0.1)


def test_forward_and_loss_match_torch_layers():
    lay = op.layout()
    theta = _theta(lay, 1)
    rng = np.random.default_rng(2)
    X = rng.normal(size=(300, 59))
    y = (rng.uniform(size=300) < 0.2).astype(np.uint8)
    w = op.unpack(theta, lay)
    f = op.mlp_forward(w, X)
    Xt = torch.tensor(X)
    h1 = torch.nn.functional.gelu(torch.nn.functional.linear(Xt, w["W1"], w["b1"]))
    h2 = torch.nn.functional.gelu(torch.nn.functional.linear(h1, w["W2"], w["b2"]))
    logit = torch.nn.functional.linear(h2, w["w3"][None], w["b3"])[:, 0]
    assert torch.allclose(f["logit"], logit, atol=1e-12, rtol=1e-12)
    for pw in (1.0, 7.5):
        ref = torch.nn.functional.binary_cross_entropy_with_logits(
            logit, torch.tensor(y, dtype=torch.float64), pos_weight=torch.tensor(pw))
        assert abs(op.bce(f["logit"], y, pw).item() - ref.item()) < 1e-13
    # the forward really uses bfloat16 weights: W1 values are bf16 grid points
    W1 = w["W1"].numpy().astype(np.float32)
    assert (op.bf16_round(W1) == W1).all()
    # and the master values differ from them
    o, n = lay["master"]["W1"]
    assert (theta[o:o + n] != W1.ravel()).mean() > 0.9


def test_gradient_matches_central_differences():
    lay = _small_layout()
    theta = _theta(lay, 5).astype(np.float64)
    rng = np.random.default_rng(6)
    X = rng.normal(size=(40, 5))
    y = (rng.uniform(size=40) < 0.4).astype(np.uint8)

    # differentiate the network at fixed (already bf16) weights: evaluate the
    # loss with the weights taken as float64 values directly
    def loss_at(th):
        w = {}
        m = lay["master"]
        for name in ("W1", "b1", "W2", "b2", "w3", "b3"):
            o, nn = m[name]
            w[name] = torch.tensor(th[o:o + nn])
        w["W1"] = w["W1"].reshape(7, 5)
        w["W2"] = w["W2"].reshape(7, 7)
        return op.bce(op.mlp_forward(w, X)["logit"], y, 3.0).item()

    # bf16-representable start so that unpack() is the identity on it
    m = lay["master"]
    th = theta.copy()
    for name in ("W1", "W2", "w3"):
        o, nn = m[name]
        th[o:o + nn] = op.bf16_round(th[o:o + nn].astype(np.float32))
    th = th.astype(np.float32).astype(np.float64)
    loss, g = op.mlp_grad(th.astype(np.float32), X, y, 3.0, lay)
    assert abs(loss - loss_at(th)) < 1e-14
    h = 1e-6
    for k in range(th.size):
        e = np.zeros_like(th)
        e[k] = h
        fd = (loss_at(th + e) - loss_at(th - e)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 + 1e-5 * abs(g[k]), (k, fd, g[k])


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(8)
    th0 = rng.normal(size=100)
    g = rng.normal(size=100)
    th1, m, v = op.adam(th0, np.zeros(100), np.zeros(100), g, 1, lr=1e-3, eps=1e-8)
    assert np.allclose(th1, th0 - 1e-3 * g / (np.abs(g) + 1e-8), atol=1e-15, rtol=1e-13)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
    # a second step with the same gradient moves by the same amount again
    th2, _, _ = op.adam(th1, m, v, g, 2, lr=1e-3, eps=1e-8)
    assert np.allclose(th2 - th1, th1 - th0, atol=1e-12)


def test_layout_sizes():
    lay = op.layout()
    assert lay["master"]["total"] == 81409
    assert lay["bf16"]["total"] == 256 * 59 + 256 * 256 + 256
    assert lay["master"]["b3"] == (81408, 1)
