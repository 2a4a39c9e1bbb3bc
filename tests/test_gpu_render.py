"""GPU parity of the render path against the FP64 oracle (tiny config and a
ragged image): records, tile keys, per-tile ranges, images, gradients."""
import math

import numpy as np
import pytest

import scenegen
from gpu_helpers import (IMG_TOL, SHAPES, assert_grad_close, check_pruned_keys,
                         flagged_pixels, gpu_render)
from oracle import splat as osp
from paper_2511_23030_amd import dcgs as D

pytestmark = pytest.mark.gpu

TILES = [(16, 16), (8, 8), (32, 16)]
SIZES = [(256, 192), (250, 190)]      # the tiny config and a ragged tail


def _scene(size, deg=0, n=10_000, seed=0):
    W, H = size
    return scenegen.tiny_scene(n=n, seed=seed, width=W, height=H, sh_degree=deg)


@pytest.mark.parametrize("size", SIZES)
@pytest.mark.parametrize("tile", TILES)
def test_keys_ranges_records(ctx, size, tile):
    sc = _scene(size)
    cam = sc["camera"]
    print(f"case keys size={size} tile={tile}", flush=True)
    g = gpu_render(ctx, sc["params"], 0, cam, [0, 0, 0], tile)
    rec = osp.preprocess(sc["params"], 0, cam, tile)
    kr = osp.tile_keys(rec)
    assert not rec.key_tie.any()
    dropped, whole = check_pruned_keys(g["keys"], g["values"], g["ranges"], g["counts"], rec, kr,
                                       what=f"size={size} tile={tile}")
    print(f"  {kr['keys'].size} oracle pairs, {dropped} left out as empty, "
          f"{whole} Gaussians left with no tile", flush=True)
    assert g["n_pairs"] == kr["keys"].size - dropped
    # records of the Gaussians the kernel draws; one it leaves with no tile
    # draws nothing (all of its pairs were shown empty above)
    vis = ~rec.culled & (g["counts"] > 0)
    assert ((g["counts"] > 0) <= ~rec.culled).all()
    assert (g["box"].T[vis] == rec.box[vis]).all()
    r = g["records"]
    u = rec.u.detach().numpy()[vis]
    v = rec.v.detach().numpy()[vis]
    assert np.abs(r[0][vis] - u).max() < 2e-5 * max(size)
    assert np.abs(r[1][vis] - v).max() < 2e-5 * max(size)
    Q = rec.conic.detach().numpy()[vis]
    for k in range(3):
        assert np.abs(r[2 + k][vis] - Q[:, k]).max() <= 1e-6 * np.abs(Q).max() + 1e-6 * np.abs(Q[:, k]).max()
    assert np.abs(r[5][vis] - rec.opacity.detach().numpy()[vis]).max() < 1e-6
    assert np.abs(r[6:9][:, vis].T - rec.rgb.detach().numpy()[vis]).max() < 1e-6
    assert (r[9][vis].astype(np.float32).view(np.int32) == rec.zbits[vis]).all()


@pytest.mark.parametrize("size", SIZES)
def test_image_parity_and_tile_independence(ctx, size):
    sc = _scene(size)
    cam = sc["camera"]
    bg = np.array([0.1, 0.2, 0.3])
    rec, img = osp.render(sc["params"], 0, cam, bg)
    flag = flagged_pixels(img)
    assert flag.sum() <= 0.001 * flag.size
    ok = ~flag
    ref_rgb = img.rgb.detach().numpy()
    imgs = []
    for shape in SHAPES:
        print(f"case image size={size} shape={shape}", flush=True)
        g = gpu_render(ctx, sc["params"], 0, cam, bg, shape[:2], ppt=shape[2])
        assert np.abs(g["rgb"] - ref_rgb)[:, ok].max() <= IMG_TOL
        assert np.abs(g["T"] - img.T.detach().numpy())[ok].max() <= IMG_TOL
        D = img.depth.detach().numpy()
        assert (np.abs(g["depth"] - D)[ok] <= IMG_TOL * np.maximum(1.0, np.abs(D[ok]))).all()
        last = g["last"]
        gid = np.where(last >= 0, g["values"][np.maximum(last, 0)], -1)
        assert (gid[ok] == img.last_g[ok]).all()
        imgs.append(g["rgb"])
    for other in imgs[1:]:
        assert (other == imgs[0]).all()          # bitwise: tile size never changes the image


@pytest.mark.parametrize("deg,size,seed,shape", [(0, (256, 192), 0, (16, 16, 2)),
                                                 (3, (250, 190), 5, (16, 16, 2)),
                                                 (0, (250, 190), 6, (16, 16, 1)),
                                                 (0, (250, 190), 7, (16, 16, 4)),
                                                 (0, (250, 190), 8, (8, 8, 1)),
                                                 (3, (250, 190), 9, (32, 16, 4)),
                                                 (0, (250, 190), 10, (32, 16, 8)),
                                                 (0, (256, 192), 11, (32, 16, 2))])
def test_gradient_parity(ctx, deg, size, seed, shape):
    sc = _scene(size, deg=deg, seed=seed)
    cam = sc["camera"]
    if deg:   # a rotated, offset camera so view directions vary
        from scipy.spatial.transform import Rotation
        R = Rotation.from_rotvec([0.05, -0.08, 0.03]).as_matrix()
        C = np.array([0.3, -0.2, -0.5])
        cam = scenegen.camera(R, -R @ C, 200.0, 200.0, size[0] / 2, size[1] / 2, size[0], size[1])
    bg = np.array([0.3, 0.1, 0.2])
    rec = osp.preprocess(sc["params"], deg, cam, requires_grad=True)
    img = osp.composite(rec, bg)
    flag = flagged_pixels(img)
    W, H = size
    dl = scenegen.upstream_grad(W, H, seed=20 + seed, scale=1e-3)
    dld = scenegen.upstream_grad(W, H, seed=30 + seed, channels=1, scale=1e-4)[0]
    dl[:, flag] = 0.0
    dld[flag] = 0.0
    gr = osp.render_grad(rec, img, dl, dld)
    print(f"case grad deg={deg} size={size} shape={shape}", flush=True)
    g = gpu_render(ctx, sc["params"], deg, cam, bg, shape[:2], dl, dld, ppt=shape[2])
    vis = ~rec.culled
    assert vis.sum() > 1000
    colour_ok = vis & (rec.raw_rgb_margin > 1e-5)
    g2 = g["grad2d"]
    assert_grad_close(g2[0:2], gr.uv.T, "d(u,v)", vis)
    assert_grad_close(g2[2:5], gr.conic.T, "d conic", vis)
    assert_grad_close(g2[5:6], gr.opacity[None], "d opacity", vis)
    assert_grad_close(g2[6:9], gr.rgb.T, "d colour", vis)
    assert_grad_close(g2[9:10], gr.z[None], "d depth", vis)
    G, Gr = g["grad"], gr.params
    assert_grad_close(G[0:3], Gr[0:3], "d mean", colour_ok)
    assert_grad_close(G[3:6], Gr[3:6], "d log-scale", vis)
    assert_grad_close(G[6:10], Gr[6:10], "d quaternion", vis)
    assert_grad_close(G[10:11], Gr[10:11], "d opacity logit", vis)
    assert_grad_close(G[11:], Gr[11:], "d SH", colour_ok)
    assert (G[:, rec.culled] == 0).all()


def test_backward_is_deterministic(ctx):
    sc = _scene((256, 192))
    cam = sc["camera"]
    dl = scenegen.upstream_grad(256, 192, seed=3, scale=1e-3)
    a = gpu_render(ctx, sc["params"], 0, cam, [0, 0, 0], (16, 16), dl)
    b = gpu_render(ctx, sc["params"], 0, cam, [0, 0, 0], (16, 16), dl)
    assert (a["grad"] == b["grad"]).all() and (a["rgb"] == b["rgb"]).all()


def test_backward_pixels_per_lane_apart_from_forward(ctx):
    # bits 4-7 of pixels_per_lane give the backward raster its own lane
    # layout: gradients then depend only on it, images on neither
    sc = _scene((256, 192))
    cam = sc["camera"]
    dl = scenegen.upstream_grad(256, 192, seed=4, scale=1e-3)
    ref = gpu_render(ctx, sc["params"], 0, cam, [0, 0, 0], (16, 16), dl, ppt=4)
    for packed in (1 | 4 << 4, 2 | 4 << 4):
        g = gpu_render(ctx, sc["params"], 0, cam, [0, 0, 0], (16, 16), dl, ppt=packed)
        assert (g["rgb"] == ref["rgb"]).all()
        assert (g["grad"] == ref["grad"]).all() and (g["grad2d"] == ref["grad2d"]).all()
    other = gpu_render(ctx, sc["params"], 0, cam, [0, 0, 0], (16, 16), dl, ppt=4 | 2 << 4)
    assert (other["rgb"] == ref["rgb"]).all()
    assert np.abs(other["grad"] - ref["grad"]).max() <= 1e-5 * np.abs(ref["grad"]).max()
    with pytest.raises(D.DcgsError):
        gpu_render(ctx, sc["params"], 0, cam, [0, 0, 0], (16, 16), dl, ppt=2 | 3 << 4)


def test_empty_and_all_culled(ctx):
    cam = scenegen.camera(np.eye(3), np.zeros(3), 50.0, 50.0, 32.0, 24.0, 64, 48)
    bg = [0.25, 0.5, 0.75]
    empty = np.zeros((14, 0), np.float32)
    g = gpu_render(ctx, empty, 0, cam, bg)
    assert (g["rgb"] == np.array(bg, np.float32)[:, None, None]).all() and (g["T"] == 1).all()
    sc = _scene((64, 48), n=500)
    p = sc["params"].copy()
    p[10] = -30.0                        # opacity below 1/255: everything culled
    dl = scenegen.upstream_grad(64, 48, seed=1)
    g = gpu_render(ctx, p, 0, cam, bg, (16, 16), dl)
    assert g["n_pairs"] == 0
    assert (g["rgb"] == np.array(bg, np.float32)[:, None, None]).all()
    assert (g["grad"] == 0).all()


def test_single_gaussian_closed_form(ctx):
    """Independent of the oracle: an isotropic Gaussian on the optical axis."""
    cam = scenegen.camera(np.eye(3), np.zeros(3), 50.0, 50.0, 32.0, 24.0, 64, 48)
    s, Z, logit = 0.05, 3.0, 0.5
    p = np.zeros((14, 1), np.float32)
    p[2, 0] = Z
    p[3:6, 0] = math.log(s)
    p[6, 0] = 1.0
    p[10, 0] = logit
    c = np.array([0.9, 0.3, 0.1])
    p[11:14, 0] = (c - 0.5) * 2 * math.sqrt(math.pi)
    bg = np.array([0.2, 0.4, 0.6])
    g = gpu_render(ctx, p, 0, cam, bg)
    var = (50.0 * s / Z) ** 2 + 0.3
    j, i = np.meshgrid(np.arange(48) + 0.5, np.arange(64) + 0.5, indexing="ij")
    a = np.minimum(0.99, np.exp(-0.5 * ((i - 32) ** 2 + (j - 24) ** 2) / var) / (1 + math.exp(-logit)))
    a = np.where(a < 1 / 255, 0.0, a)
    assert np.abs(g["rgb"] - (c[:, None, None] * a + (1 - a) * bg[:, None, None])).max() < IMG_TOL


def test_keys_rotated_camera_sh3(ctx):
    """A rotated, offset camera: keys and ranges bit-exact on every tile whose
    list holds no Gaussian within 1e-11 of a rounding or integer decision;
    a flagged Gaussian's depth key is one of the two nearest float32 values."""
    from scipy.spatial.transform import Rotation
    sc = _scene((250, 190), deg=3, seed=5)
    R = Rotation.from_rotvec([0.05, -0.08, 0.03]).as_matrix()
    C = np.array([0.3, -0.2, -0.5])
    cam = scenegen.camera(R, -R @ C, 200.0, 200.0, 125.0, 95.0, 250, 190)
    g = gpu_render(ctx, sc["params"], 3, cam, [0, 0, 0], (16, 16))
    rec = osp.preprocess(sc["params"], 3, cam, (16, 16))
    kr = osp.tile_keys(rec)
    tie = rec.key_tie
    assert tie.sum() <= 10
    zg = g["records"][9].astype(np.float32).view(np.int32).astype(np.int64)
    drawn = g["counts"] > 0
    assert (np.abs(zg[tie & drawn] - rec.zbits[tie & drawn]) <= 1).all()
    dropped, whole = check_pruned_keys(g["keys"], g["values"], g["ranges"], g["counts"], rec, kr,
                                       tie=tie, what="rotated camera SH3")
    print(f"  {kr['keys'].size} oracle pairs, {dropped} left out as empty, {whole} Gaussians "
          f"left with no tile, {tie.sum()} key ties", flush=True)
