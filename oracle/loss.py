"""Oracle: the paper's mapping loss, Eqs. (2)-(4), in float64.

TEST INFRASTRUCTURE ONLY (see the package header).

    L = L_image + lambda_depth L_depth                        (Eq. 2)
    L_image = (1 - lambda_s) |I - I_gt|_1 + lambda_s (1 - SSIM(I, I_gt))   (Eq. 3)
    L_depth = |D_r - D_gt|_1                                  (Eq. 4)

Readings (the paper names SSIM and the norms, not their constants):

* |.|_1 is the mean absolute difference over the 3HW colour values (HW
  depth values for Eq. 4);
* SSIM is the mean over the 3HW values of the usual per-pixel structural
  similarity with an 11-tap Gaussian window of standard deviation 1.5
  (normalised to sum 1, applied separably), zero padding outside the image
  ("same" size), C1 = 0.01^2, C2 = 0.03^2, each colour channel on its own:
  S = ((2 mx my + C1) (2 sxy + C2)) / ((mx^2 + my^2 + C1) (sx + sy + C2))
  with mx = G*x, sx = G*(x^2) - mx^2, sxy = G*(x y) - mx my;
* a window of V views sums the per-view losses.

What pins each function (tests/test_oracle_loss.py):

* ``gaussian_window``  scipy.signal.windows.gaussian, normalised.
* ``blur``             brute-force loops on small images.
* ``ssim_map``         SSIM(x, x) = 1; constant images in closed form away
                       from the border; symmetry in (x, y).
* ``mapping_loss``     lambda_s = 0 and 1 and lambda_depth = 0 reduce to its
                       terms; the gradient against central finite
                       differences.
"""
from __future__ import annotations

import math

import numpy as np
import torch

C1 = 0.01 ** 2
C2 = 0.03 ** 2
WINDOW = 11
SIGMA = 1.5


def gaussian_window(size: int = WINDOW, sigma: float = SIGMA) -> torch.Tensor:
    k = torch.arange(size, dtype=torch.float64) - (size - 1) / 2.0
    g = torch.exp(-(k * k) / (2.0 * sigma * sigma))
    return g / g.sum()


def blur(img: torch.Tensor, size: int = WINDOW, sigma: float = SIGMA) -> torch.Tensor:
    """Separable Gaussian blur of [..., H, W] planes, zero padding, same size."""
    g = gaussian_window(size, sigma)
    shape = img.shape
    x = img.reshape(-1, 1, shape[-2], shape[-1])
    x = torch.nn.functional.conv2d(x, g.view(1, 1, 1, size), padding=(0, size // 2))
    x = torch.nn.functional.conv2d(x, g.view(1, 1, size, 1), padding=(size // 2, 0))
    return x.reshape(shape)


def ssim_map(x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    mx, my = blur(x), blur(y)
    sx = blur(x * x) - mx * mx
    sy = blur(y * y) - my * my
    sxy = blur(x * y) - mx * my
    return ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sx + sy + C2))


def mapping_loss(rgb, target, depth=None, depth_target=None, lambda_s: float = 0.2,
                 lambda_depth: float = 0.0) -> torch.Tensor:
    """Eq. (2) summed over views: rgb, target [V, 3, H, W]; depth,
    depth_target [V, H, W] (needed when lambda_depth != 0)."""
    rgb = torch.as_tensor(rgb, dtype=torch.float64)
    target = torch.as_tensor(target, dtype=torch.float64)
    if rgb.dim() == 3:
        rgb, target = rgb[None], target[None]
    total = rgb.new_zeros(())
    for v in range(rgb.shape[0]):
        l1 = (rgb[v] - target[v]).abs().mean()
        img = (1.0 - lambda_s) * l1
        if lambda_s != 0.0:
            img = img + lambda_s * (1.0 - ssim_map(rgb[v], target[v]).mean())
        total = total + img
        if lambda_depth != 0.0:
            d = torch.as_tensor(depth, dtype=torch.float64)
            dt = torch.as_tensor(depth_target, dtype=torch.float64)
            if d.dim() == 2:
                d, dt = d[None], dt[None]
            total = total + lambda_depth * (d[v] - dt[v]).abs().mean()
    return total


def mapping_loss_grad(rgb, target, depth=None, depth_target=None, lambda_s: float = 0.2,
                      lambda_depth: float = 0.0):
    """(loss, dL/drgb, dL/ddepth or None) by reverse-mode differentiation."""
    x = torch.tensor(np.asarray(rgb, np.float64), requires_grad=True)
    d = None
    if depth is not None:
        d = torch.tensor(np.asarray(depth, np.float64), requires_grad=True)
    L = mapping_loss(x, target, d, depth_target, lambda_s, lambda_depth)
    L.backward()
    return float(L.detach()), x.grad.numpy(), (d.grad.numpy() if d is not None and
                                               d.grad is not None else None)


def psnr(mse: float) -> float:
    return 10.0 * math.log10(1.0 / mse)
