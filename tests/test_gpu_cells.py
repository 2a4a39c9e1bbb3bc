"""The rasterizers skip 8x8 cells that a record's pixel box or alpha >= 1/255
ellipse cannot reach.  A stress scene of needle-like Gaussians at every
angle (axis ratios up to ~1e3, so conics up to ~1e6 in condition number,
many too ill-conditioned for the ellipse test to decide) with opacities
close to the 1/255 threshold must render identically, bit for bit, with
every raster shape: the 8x8 tile (one cell, no cell masks) against the
multi-cell ones.  The backward is checked on terms that are sums of
non-negative contributions (a constant positive upstream gradient makes a
record's colour and depth terms sums of weights), so float32 summation in
another order agrees to ~1e-5 while a skipped cell would drop whole pixel
contributions; gradients with cancelling terms are compared with the FP64
oracle elsewhere."""
import numpy as np
import pytest

import scenegen
from gpu_helpers import SHAPES, gpu_render

pytestmark = pytest.mark.gpu

ROW_LOG_SCALE, ROW_OPACITY = 3, 10


def _needles(size, seed):
    W, H = size
    sc = scenegen.tiny_scene(n=3000, seed=seed, width=W, height=H, sh_degree=0)
    P = sc["params"].astype(np.float64)
    rng = np.random.default_rng(seed + 100)
    n = P.shape[1]
    # one long axis, two very short ones
    P[ROW_LOG_SCALE] = rng.uniform(-2.0, 0.3, n)
    P[ROW_LOG_SCALE + 1] = rng.uniform(-7.5, -5.0, n)
    P[ROW_LOG_SCALE + 2] = rng.uniform(-7.5, -5.0, n)
    # half of them just above the alpha threshold, the rest ordinary
    o = rng.uniform(1.0 / 255.0, 0.03, n)
    near = rng.uniform(size=n) < 0.5
    P[ROW_OPACITY] = np.where(near, np.log(o / (1.0 - o)), rng.normal(0.0, 1.0, n))
    sc["params"] = P.astype(np.float32)
    return sc


@pytest.mark.parametrize("size,seed", [((256, 192), 3), ((250, 190), 4)])
def test_needles_render_identically_with_every_raster_shape(ctx, size, seed):
    sc = _needles(size, seed)
    cam = sc["camera"]
    bg = np.array([0.2, 0.1, 0.3])
    W, H = size
    dl = np.full((3, H, W), 1e-3, np.float32)
    dld = np.full((H, W), 1e-4, np.float32)
    print(f"case needles size={size} seed={seed} shape=(8, 8, 1)", flush=True)
    ref = gpu_render(ctx, sc["params"], 0, cam, bg, (8, 8), dl=dl, dld=dld, ppt=1)
    assert ref["n_pairs"] > 0 and (ref["T"] < 1.0).mean() > 0.05
    r2 = ref["grad2d"][6:10].astype(np.float64)
    assert (r2 >= 0).all() and (r2 > 0).any()
    for shape in SHAPES:
        if shape == (8, 8, 1):
            continue
        print(f"case needles size={size} seed={seed} shape={shape}", flush=True)
        g = gpu_render(ctx, sc["params"], 0, cam, bg, shape[:2], dl=dl, dld=dld, ppt=shape[2])
        assert (g["rgb"] == ref["rgb"]).all()
        assert (g["depth"] == ref["depth"]).all()
        assert (g["T"] == ref["T"]).all()
        g2 = g["grad2d"][6:10].astype(np.float64)
        err = np.abs(g2 - r2)
        assert (err <= 2e-4 * r2 + 1e-30).all(), (shape, float((err / np.maximum(r2, 1e-30)).max()))
