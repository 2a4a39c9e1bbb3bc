"""torch.autograd through the hand-written adjoint, against FP64 finite
differences of the oracle's forward along random directions (a 1,000-
Gaussian subset of the tiny scene, SH degree 3)."""
import math

import numpy as np
import pytest
import torch

import scenegen
from oracle import splat as osp
from paper_2511_23030_amd.render import render

pytestmark = pytest.mark.gpu


def test_autograd_matches_directional_fd(ctx):
    sc = scenegen.tiny_scene(n=1000, seed=40, width=96, height=72, focal=80.0, sh_degree=3)
    cam = sc["camera"]
    bg = np.array([0.2, 0.3, 0.4])
    P = sc["params"].astype(np.float64)
    rec, img = osp.render(P, 3, cam, bg)
    flag = ((img.margin_alpha < 1e-3) | (img.margin_T < 1e-3) | (img.margin_clamp < 1e-3))
    rng = np.random.default_rng(41)
    w = rng.normal(size=(3, 72, 96))
    w[:, flag] = 0.0
    wd = rng.normal(size=(72, 96)) * 0.05
    wd[flag] = 0.0
    Pt = torch.tensor(sc["params"], device="cuda", requires_grad=True)
    rgb, depth = render(Pt, ctx, cam, bg, 3)
    loss = (rgb * torch.tensor(w, dtype=torch.float32, device="cuda")).sum() + \
        (depth * torch.tensor(wd, dtype=torch.float32, device="cuda")).sum()
    loss.backward()
    g = Pt.grad.cpu().numpy().astype(np.float64)
    assert np.isfinite(g).all() and np.abs(g).max() > 0

    def objective(Q):
        _, im = osp.render(Q, 3, cam, bg)
        return float((im.rgb.detach().numpy() * w).sum() + (im.depth.detach().numpy() * wd).sum())

    vis = ~rec.culled & (rec.raw_rgb_margin > 1e-4)
    for k in range(8):
        d = rng.normal(size=P.shape) * vis[None, :]
        d /= np.linalg.norm(d)
        h = 1e-6
        fd = (objective(P + h * d) - objective(P - h * d)) / (2 * h)
        ad = float((g * d).sum())
        assert abs(fd - ad) <= 1e-3 * max(abs(fd), 1e-3 * np.linalg.norm(g)), (k, fd, ad)
