"""The LoG sampling map on the GPU against the FP64 oracle: the map within
float32 accuracy, the selected pixel list exact away from ties."""
import numpy as np
import pytest
import torch

import scenegen
from oracle import sampling as osm

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("H,W,sigma", [(16, 16, 1.0), (37, 53, 1.0), (96, 128, 1.5),
                                       (180, 320, 2.0)])
def test_sampling_map_and_selection(ctx, H, W, sigma):
    rng = np.random.default_rng(H + W)
    image = rng.uniform(size=(3, H, W)).astype(np.float32)
    # a render with the same coarse structure and less detail
    render = np.clip(image + rng.normal(0, 0.05, size=image.shape), 0, 1).astype(np.float32)
    u = scenegen.target_image(W, H, seed=H, channels=1)[0]
    ps, idx = ctx.sample_pixels(torch.from_numpy(image).cuda(), torch.from_numpy(render).cuda(),
                                torch.from_numpy(u).cuda(), beta=2.0, sigma=sigma)
    ref = osm.sampling_map(image.astype(np.float64), render.astype(np.float64), 2.0, sigma)
    assert np.abs(ps.cpu().numpy() - ref).max() <= 1e-5
    sel, ties = osm.sample_pixels(image.astype(np.float64), render.astype(np.float64),
                                  u.astype(np.float64), 2.0, sigma)
    got = idx.cpu().numpy()
    assert (np.diff(got) > 0).all()
    keep = ~ties.ravel()
    mask_got = np.zeros(H * W, bool)
    mask_got[got] = True
    mask_ref = np.zeros(H * W, bool)
    mask_ref[sel] = True
    assert (mask_got[keep] == mask_ref[keep]).all()
    assert mask_ref.sum() > 0


def test_identical_images_sample_nothing(ctx):
    rng = np.random.default_rng(3)
    image = torch.from_numpy(rng.uniform(size=(3, 40, 60)).astype(np.float32)).cuda()
    u = torch.zeros(40, 60, device="cuda")
    ps, idx = ctx.sample_pixels(image, image.clone(), u)
    assert ps.abs().max().item() == 0.0 and idx.numel() == 0
