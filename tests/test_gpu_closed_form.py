"""Closed-form cases run on the GPU (the same cases pin the oracle): the
termination of a stack of alpha = 1/2 Gaussians with tied depths, and the
0.99 clamp, through every raster shape."""
import math

import numpy as np
import pytest
import torch

from gpu_helpers import SHAPES, gpu_render
from test_oracle_splat import CAM, make_params

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape", SHAPES)
def test_stack_of_thirteen_terminates_with_ties_in_index_order(ctx, shape):
    """16 identical Gaussians with alpha = 1/2 exactly at the centre of pixel
    (32, 24) (opacity 1/2, the pixel centre on the mean): T = 2^-k after k
    of them, and 2^-14 < 1e-4 <= 2^-13, so exactly 13 are composited; their
    depths are equal, so the 13th in list order is Gaussian 12."""
    bg = np.array([0.0, 0.5, 1.0])
    c = np.array([0.8, 0.6, 0.4])
    Z = 3.0
    X = 0.5 * Z / 50.0
    P = make_params([[X, X, Z]] * 16, [math.log(0.05)] * 3, [1, 0, 0, 0], 0.0, c)
    out = gpu_render(ctx, P.astype(np.float32), 0, CAM, bg, shape[:2], ppt=shape[2])
    t = 2.0 ** -13
    assert abs(float(out["T"][24, 32]) - t) <= 1e-6 * t
    last = int(out["last"][24, 32])
    assert out["values"][last] == 12
    # the 13 composited are Gaussians 0..12, in index order, at the head of
    # the list of the pixel's tile
    tiles_x = (64 + shape[0] - 1) // shape[0]
    lo = int(out["ranges"][(24 // shape[1]) * tiles_x + 32 // shape[0]][0])
    assert out["values"][lo:last + 1].tolist() == list(range(13))
    ref = c * (1 - t) + bg * t
    assert np.abs(out["rgb"][:, 24, 32] - ref).max() <= 1e-6


@pytest.mark.parametrize("shape", [(16, 16, 2), (8, 8, 1), (32, 16, 8)])
def test_clamp_at_099_passes_no_opacity_or_position_gradient(ctx, shape):
    """One Gaussian whose o G exceeds 0.99 at the centre of pixel (32, 24):
    alpha is clamped to 0.99 there, so T = 1 - 0.99 and C = 0.99 c, and a
    loss on that pixel alone sends no gradient to the opacity or the
    position (the clamp's derivative is 0)."""
    c = np.array([0.3, 0.6, 0.9])
    Z = 2.0
    P = make_params([[0.5 * Z / 50.0, 0.5 * Z / 50.0, Z]], [math.log(0.05)] * 3, [1, 0, 0, 0],
                    10.0, c)
    dl = np.zeros((3, 48, 64), np.float32)
    dl[:, 24, 32] = 1.0
    out = gpu_render(ctx, P.astype(np.float32), 0, CAM, np.zeros(3), shape[:2], dl=dl,
                     ppt=shape[2])
    a = np.float32(0.99)
    assert abs(float(out["T"][24, 32]) - (1.0 - float(a))) <= 1e-7
    assert np.abs(out["rgb"][:, 24, 32] - a * c.astype(np.float32)).max() <= 1e-7
    g2 = out["grad2d"][:, 0]                 # (u, v, Q00, Q01, Q11, o, r, g, b, Z)
    assert g2[0] == 0.0 and g2[1] == 0.0 and g2[5] == 0.0
    assert g2[2] == 0.0 and g2[3] == 0.0 and g2[4] == 0.0
    assert out["grad"][10, 0] == 0.0         # opacity logit
    # the colour still receives alpha T = 0.99 per channel
    assert np.abs(g2[6:9] - a).max() <= 1e-6
