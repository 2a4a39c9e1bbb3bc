"""Oracle: the LoG sampling map of the Sampling section, in float64.

TEST INFRASTRUCTURE ONLY (see the package header).

For each keyframe the paper draws new primitives where the image has detail
the current reconstruction lacks:

    P_s(x, y) = max(P_L(x, y) - P~(x, y), 0)          (the sampling equation)

with P_L from the Laplacian-of-Gaussian (LoG) response of the input image
and P~ from that of the rendered image.  Readings (the paper defers the
constants to prior work):

* the LoG is scipy's gaussian_laplace: the sum of the second-derivative
  Gaussian filters along rows and along columns, sigma = 1 px, kernel
  radius ceil(4 sigma), the 1D kernels the sampled, normalised Gaussian and
  its exact second derivative, mirror ("reflect", edge sample repeated)
  boundary;
* the response of a colour image is the Euclidean norm over its three
  channels of the per-channel LoG;
* P_L = min(1, beta * response of the input), P~ = min(1, beta * response
  of the render), beta = 2 by default;
* a pixel is sampled when a uniform number u(x, y) drawn for it (an input)
  is below P_s(x, y); the sampled pixels are listed in raster order.

What pins each function (tests/test_oracle_sampling.py):

* ``log_kernels``   the second-derivative kernel against the analytic
                    derivative of the sampled Gaussian; zero-sum of the
                    second derivative of a symmetric quadratic.
* ``log_response``  brute-force 2D convolution with reflect padding; a linear
                    image has zero response away from the border.
* ``sampling_map`` / ``sample_pixels``  identical images give P_s = 0; a
                    flat render gives P_s = P_L; brute-force selection.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.ndimage

SIGMA = 1.0
BETA = 2.0


def log_kernels(sigma: float = SIGMA) -> tuple:
    """1D Gaussian (normalised) and its second derivative, radius ceil(4 sigma)."""
    r = int(math.ceil(4.0 * sigma))
    x = np.arange(-r, r + 1, dtype=np.float64)
    g = np.exp(-0.5 * x * x / (sigma * sigma))
    g /= g.sum()
    d2 = (x * x / sigma ** 4 - 1.0 / sigma ** 2) * g
    return g, d2


def log_response(img, sigma: float = SIGMA) -> np.ndarray:
    """Euclidean norm over channels of the per-channel LoG; img [C, H, W]."""
    img = np.asarray(img, np.float64)
    lap = np.stack([scipy.ndimage.gaussian_laplace(img[c], sigma, mode="reflect")
                    for c in range(img.shape[0])])
    return np.sqrt((lap * lap).sum(0))


def sampling_map(image, render, beta: float = BETA, sigma: float = SIGMA) -> np.ndarray:
    pl = np.minimum(1.0, beta * log_response(image, sigma))
    pt = np.minimum(1.0, beta * log_response(render, sigma))
    return np.maximum(pl - pt, 0.0)


def sample_pixels(image, render, u, beta: float = BETA, sigma: float = SIGMA,
                  tie: float = 1e-5) -> tuple:
    """Raster-order indices of the sampled pixels and a mask of pixels whose
    u lies within `tie` of P_s (float32 evaluation may decide them either
    way)."""
    ps = sampling_map(image, render, beta, sigma)
    u = np.asarray(u, np.float64)
    sel = np.flatnonzero((u < ps).ravel())
    ties = np.abs(u - ps) <= tie
    return sel, ties
