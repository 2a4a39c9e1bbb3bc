"""Pins of the splatting oracle: closed forms, brute force, finite differences."""
import math

import numpy as np
from scipy.spatial.transform import Rotation
import pytest
import torch

import scenegen
from oracle import splat as osp

Y00 = 1.0 / (2.0 * math.sqrt(math.pi))


def make_params(means, log_scale, quat, logit, rgb, deg=0, rest=None):
    """Parameter block for n Gaussians; log_scale/quat/rgb are either one row
    shared by all Gaussians or one row per Gaussian."""
    means = np.atleast_2d(np.asarray(means, np.float64))
    n = means.shape[0]

    def rows(x, k):
        x = np.asarray(x, np.float64)
        return np.broadcast_to(x.reshape(-1, k), (n, k)).T
    P = np.zeros((11 + 3 * (deg + 1) ** 2, n))
    P[0:3] = means.T
    P[3:6] = rows(log_scale, 3)
    P[6:10] = rows(quat, 4)
    P[10] = logit
    P[11:14] = (rows(rgb, 3) - 0.5) / Y00
    if rest is not None:
        P[14:] = rest
    return P


CAM = scenegen.camera(np.eye(3), np.zeros(3), 50.0, 50.0, 32.0, 24.0, 64, 48)


def pixel_grid(W, H):
    j, i = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    return i + 0.5, j + 0.5


def test_single_isotropic_on_axis_closed_form():
    s, Z, logit = 0.05, 3.0, 0.5
    c = np.array([0.9, 0.3, 0.1])
    bg = np.array([0.2, 0.4, 0.6])
    P = make_params([[0.0, 0.0, Z]], [math.log(s)] * 3, [1, 0, 0, 0], logit, c)
    rec, img = osp.render(P, 0, CAM, bg)
    o = 1 / (1 + math.exp(-logit))
    var = (50.0 * s / Z) ** 2 + 0.3            # on the axis J = diag(f/Z, f/Z)
    px, py = pixel_grid(64, 48)
    a = np.minimum(0.99, o * np.exp(-0.5 * ((px - 32) ** 2 + (py - 24) ** 2) / var))
    a = np.where(a < 1 / 255, 0.0, a)
    exp_rgb = c[:, None, None] * a + (1 - a) * bg[:, None, None]
    assert np.abs(img.rgb.detach().numpy() - exp_rgb).max() < 1e-12
    assert np.abs(img.T.detach().numpy() - (1 - a)).max() < 1e-12
    assert np.abs(img.depth.detach().numpy() - Z * a).max() < 1e-12
    assert (img.n_contrib == (a > 0)).all()


def _fd_jacobian(cam, Xc, h=1e-6):
    def proj(X):
        return np.array([cam["fx"] * X[0] / X[2] + cam["cx"], cam["fy"] * X[1] / X[2] + cam["cy"]])
    J = np.zeros((2, 3))
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        J[:, k] = (proj(Xc + e) - proj(Xc - e)) / (2 * h)
    return J


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_single_isotropic_off_axis_fd_jacobian(seed):
    """An isotropic Gaussian anywhere, under any camera rotation: Sigma2 =
    s^2 J J^T + 0.3 I with J the finite-difference Jacobian of the pinhole map."""
    rng = np.random.default_rng(seed)
    cam = scenegen.random_cameras(1, seed=100 + seed, extent=0.0, width=64, height=48, focal=50.0)[0]
    cam["z_far"] = 100.0
    Xc = np.array([rng.uniform(-0.8, 0.8), rng.uniform(-0.6, 0.6), rng.uniform(2.0, 4.0)])
    mu = cam["R"].T @ (Xc - cam["t"])
    s = 0.06
    q = rng.normal(size=4)
    P = make_params([mu], [math.log(s)] * 3, q, 1.0, [0.7, 0.2, 0.5])
    rec, img = osp.render(P, 0, cam, np.zeros(3))
    J = _fd_jacobian(cam, Xc)
    S2 = s * s * J @ J.T + 0.3 * np.eye(2)
    Q = np.linalg.inv(S2)
    u = cam["fx"] * Xc[0] / Xc[2] + cam["cx"]
    v = cam["fy"] * Xc[1] / Xc[2] + cam["cy"]
    px, py = pixel_grid(64, 48)
    dx, dy = px - u, py - v
    o = 1 / (1 + math.exp(-1.0))
    a = np.minimum(0.99, o * np.exp(-0.5 * (Q[0, 0] * dx * dx + 2 * Q[0, 1] * dx * dy + Q[1, 1] * dy * dy)))
    a = np.where(a < 1 / 255, 0.0, a)
    assert np.abs(img.T.detach().numpy() - (1 - a)).max() < 1e-6


def test_zero_opacity_is_background_exactly():
    bg = np.array([0.25, 0.5, 0.75])
    P = make_params([[0.0, 0.0, 3.0], [0.1, 0.0, 2.5]], [math.log(0.1)] * 3, [1, 0, 0, 0], -30.0, [0.9, 0.1, 0.2])
    rec = osp.preprocess(P, 0, CAM, requires_grad=True)
    assert rec.culled.all()
    img = osp.composite(rec, bg)
    assert (img.rgb.detach().numpy() == bg[:, None, None]).all()
    assert (img.T.detach().numpy() == 1.0).all() and (img.depth.detach().numpy() == 0.0).all()
    gr = osp.render_grad(rec, img, np.ones((3, 48, 64)), np.ones((48, 64)))
    assert (gr.params == 0.0).all()


def test_two_gaussians_closed_form():
    bg = np.array([0.1, 0.2, 0.3])
    c1, c2 = np.array([1.0, 0.0, 0.5]), np.array([0.0, 1.0, 0.25])
    s1, s2, Z1, Z2 = 0.05, 0.08, 2.0, 3.5
    P = make_params([[0.0, 0.0, Z2], [0.0, 0.0, Z1]], [[math.log(s2)] * 3, [math.log(s1)] * 3],
                    [1, 0, 0, 0], np.array([0.3, -0.2]), np.stack([c2, c1]))
    rec, img = osp.render(P, 0, CAM, bg)
    px, py = pixel_grid(64, 48)
    r2 = (px - 32) ** 2 + (py - 24) ** 2

    def alpha(s, Z, logit):
        var = (50.0 * s / Z) ** 2 + 0.3
        a = np.minimum(0.99, np.exp(-0.5 * r2 / var) / (1 + math.exp(-logit)))
        return np.where(a < 1 / 255, 0.0, a)
    a1, a2 = alpha(s1, Z1, -0.2), alpha(s2, Z2, 0.3)     # Gaussian 1 (index 1) is in front
    exp_rgb = (c1[:, None, None] * a1 + c2[:, None, None] * a2 * (1 - a1)
               + bg[:, None, None] * (1 - a1) * (1 - a2))
    assert np.abs(img.rgb.detach().numpy() - exp_rgb).max() < 1e-12
    assert np.abs(img.depth.detach().numpy() - (Z1 * a1 + Z2 * a2 * (1 - a1))).max() < 1e-12


def test_termination_stack_of_thirteen():
    """16 identical Gaussians with alpha = 1/2 at a pixel centre: T = 2^-k
    after k, and 2^-14 < 1e-4 <= 2^-13, so exactly 13 are composited."""
    bg = np.array([0.0, 0.5, 1.0])
    c = np.array([0.8, 0.6, 0.4])
    Z = 3.0
    X = 0.5 * Z / 50.0                       # u = 32.5: centre of pixel column 32
    P = make_params([[X, 0.5 * Z / 50.0, Z]] * 16, [math.log(0.05)] * 3, [1, 0, 0, 0], 0.0, c)
    rec, img = osp.render(P, 0, CAM, bg)
    assert img.n_contrib[24, 32] == 13
    assert img.last_g[24, 32] == 12           # equal depths: ascending index
    t = 2.0 ** -13
    assert abs(img.T[24, 32].item() - t) < 1e-15
    assert np.abs(img.rgb[:, 24, 32].detach().numpy() - (c * (1 - t) + bg * t)).max() < 1e-12


def test_clamp_at_099():
    c = np.array([0.3, 0.6, 0.9])
    Z = 2.0
    P = make_params([[0.5 * Z / 50.0, 0.5 * Z / 50.0, Z]], [math.log(0.05)] * 3, [1, 0, 0, 0], 10.0, c)
    rec = osp.preprocess(P, 0, CAM, requires_grad=True)
    img = osp.composite(rec, np.zeros(3))
    assert abs(img.T[24, 32].item() - 0.01) < 1e-15
    assert np.abs(img.rgb[:, 24, 32].detach().numpy() - 0.99 * c).max() < 1e-15
    w = np.zeros((3, 48, 64))
    w[:, 24, 32] = 1.0
    gr = osp.render_grad(rec, img, w)
    assert gr.params[10, 0] == 0.0           # clamped alpha passes no gradient to o
    assert gr.uv[0, 0] == 0.0


def test_box_holds_every_visible_sample():
    sc = scenegen.tiny_scene(n=3000, seed=4)
    rec = osp.preprocess(sc["params"], 0, sc["camera"])
    W, H = sc["camera"]["width"], sc["camera"]["height"]
    px, py = pixel_grid(W, H)
    idx = np.nonzero(~rec.culled)[0][:300]
    u, v = rec.u.detach().numpy(), rec.v.detach().numpy()
    Q, o = rec.conic.detach().numpy(), rec.opacity.detach().numpy()
    for g in idx:
        dx, dy = px - u[g], py - v[g]
        a = o[g] * np.exp(-0.5 * (Q[g, 0] * dx * dx + Q[g, 2] * dy * dy) - Q[g, 1] * dx * dy)
        jj, ii = np.nonzero(a >= 1 / 255)
        i0, i1, j0, j1 = rec.box[g]
        assert ((ii >= i0) & (ii <= i1) & (jj >= j0) & (jj <= j1)).all()
        # and the box is tight: its edge columns/rows hold a sample near the cutoff
        assert len(ii) > 0


def _rect_tiles(rec):
    """{(g, tx, ty)} of every tile of every drawn Gaussian's tile rectangle."""
    out = set()
    for g in np.nonzero(~rec.culled)[0]:
        tx0, tx1, ty0, ty1 = rec.tile_rect[g]
        for ty in range(ty0, ty1 + 1):
            for tx in range(tx0, tx1 + 1):
                out.add((g, tx, ty))
    return out


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 16)])
def test_keys_and_ranges_linear_scan(tile):
    sc = scenegen.tiny_scene(n=400, seed=6, width=70, height=50, focal=60.0)
    rec = osp.preprocess(sc["params"], 0, sc["camera"], tile=tile)
    kr = osp.tile_keys(rec)
    pairs = _rect_tiles(rec)
    nt = kr["tiles_x"] * kr["tiles_y"]
    for t in range(nt):
        tx, ty = t % kr["tiles_x"], t // kr["tiles_x"]
        lst = [g for g in range(400) if (g, tx, ty) in pairs]
        lst.sort(key=lambda g: (rec.zbits[g], g))
        lo, hi = kr["ranges"][t]
        assert list(kr["values"][lo:hi]) == lst
        assert all(int(k) >> 32 == t for k in kr["keys"][lo:hi])
        assert (kr["tx"][lo:hi] == tx).all() and (kr["ty"][lo:hi] == ty).all()
    assert kr["counts"].sum() == len(pairs) == kr["keys"].size


@pytest.mark.parametrize("tile", [(16, 16), (8, 8)])
def test_every_alpha_sample_lies_in_a_binned_tile(tile):
    """Brute force over every pixel of the image: a (pixel, Gaussian) sample
    with alpha >= 1/255 lies in one of the Gaussian's binned tiles."""
    sc = scenegen.tiny_scene(n=3000, seed=4)
    cam = sc["camera"]
    rec = osp.preprocess(sc["params"], 0, cam, tile)
    pairs = _rect_tiles(rec)
    W, H = cam["width"], cam["height"]
    px, py = pixel_grid(W, H)
    u, v = rec.u.detach().numpy(), rec.v.detach().numpy()
    Q, o = rec.conic.detach().numpy(), rec.opacity.detach().numpy()
    for g in np.nonzero(~rec.culled)[0][:400]:
        dx, dy = px - u[g], py - v[g]
        a = o[g] * np.exp(-0.5 * (Q[g, 0] * dx * dx + Q[g, 2] * dy * dy) - Q[g, 1] * dx * dy)
        jj, ii = np.nonzero(a >= 1 / 255)
        for tx, ty in set(zip(ii // tile[0], jj // tile[1])):
            assert (g, tx, ty) in pairs


def test_pair_alpha_max_isotropic_closed_form():
    """One isotropic Gaussian at u = 32.3, v = 24.2 (continuous pixel
    coordinates) under 8x8 tiles: the largest alpha of a tile is at its pixel
    centre nearest to (u, v), o exp(-r^2 / (2 var)) with var = (f s/Z)^2 + 0.3;
    a tile the box misses reports -inf."""
    Z, s, logit = 3.0, 0.08, 1.0
    u0, v0 = 32.3, 24.2
    # on the optical axis (J = diag(f/Z, f/Z) exactly), principal point at (u0, v0)
    cam = scenegen.camera(np.eye(3), np.zeros(3), 50.0, 50.0, u0, v0, 64, 48)
    P = make_params([[0.0, 0.0, Z]], [math.log(s)] * 3, [1, 0, 0, 0], logit, [0.5, 0.5, 0.5])
    rec = osp.preprocess(P, 0, cam, (8, 8))
    o = 1 / (1 + math.exp(-logit))
    var = (50.0 * s / Z) ** 2 + 0.3
    # tile (4, 3) holds pixel (32, 24), centre (32.5, 24.5); the tile to its
    # left ends at column 31 (centre 31.5); the one above ends at row 23
    cases = {(4, 3): (0.2, 0.3), (3, 3): (0.8, 0.3), (4, 2): (0.2, 0.7), (3, 2): (0.8, 0.7),
             (5, 3): (8.2, 0.3)}
    g = np.zeros(len(cases), np.int64)
    tx = np.array([c[0] for c in cases])
    ty = np.array([c[1] for c in cases])
    got = osp.pair_alpha_max(rec, g, tx, ty)
    for k, (dx, dy) in enumerate(cases.values()):
        exp = o * math.exp(-0.5 * (dx * dx + dy * dy) / var)
        i0, i1, j0, j1 = rec.box[0]
        in_box = (tx[k] * 8 + 7 >= i0) and (tx[k] * 8 <= i1) and (ty[k] * 8 + 7 >= j0) and (ty[k] * 8 <= j1)
        if in_box:
            assert abs(got[k] - exp) <= 1e-12, (k, got[k], exp)
        else:
            assert got[k] == -np.inf
    # the far tile (5, 3) lies beyond the box of this small Gaussian
    assert got[4] == -np.inf and rec.box[0][1] < 40


@pytest.mark.parametrize("seed", [0, 1])
def test_pair_alpha_max_against_one_gaussian_renders(seed):
    """Each Gaussian composited alone: its transmittance is 1 - alpha where it
    draws and 1 elsewhere, so over a tile the largest 1 - T equals the pair's
    alpha maximum (clamped at 0.99) when that reaches 1/255, and the tile is
    untouched (T = 1) when it does not."""
    sc = scenegen.tiny_scene(n=60, seed=30 + seed, width=64, height=48, focal=50.0)
    cam = sc["camera"]
    rec = osp.preprocess(sc["params"], 0, cam, (8, 8))
    kr = osp.tile_keys(rec)
    got = osp.pair_alpha_max(rec, kr["values"], kr["tx"], kr["ty"])
    assert (got > -np.inf).all()            # every rectangle tile meets the box
    below = 0
    for k, g in enumerate(kr["values"]):
        one = osp.preprocess(sc["params"][:, [g]], 0, cam, (8, 8))
        img = osp.composite(one, np.zeros(3))
        tx, ty = kr["tx"][k], kr["ty"][k]
        Tt = img.T.detach().numpy()[ty * 8:ty * 8 + 8, tx * 8:tx * 8 + 8]
        if got[k] >= 1 / 255:
            assert abs((1 - Tt.min()) - min(0.99, got[k])) <= 1e-12
        else:
            assert (Tt == 1.0).all()
            below += 1
    assert below > 0                        # some rectangle tiles hold no sample


def _fd_scene(seed, deg=3, n=40):
    rng = np.random.default_rng(seed)
    cam = scenegen.look_camera([0.0, 0.0, 0.0], 0.3, -0.1, 50.0, 55.0, 64, 48, 0.2, 50.0)
    R, t = cam["R"], cam["t"]
    Xc = np.stack([rng.uniform(-0.9, 0.9, n), rng.uniform(-0.6, 0.6, n), rng.uniform(2.0, 4.0, n)], 1)
    mu = (Xc - t) @ R
    P = np.zeros((11 + 3 * (deg + 1) ** 2, n))
    P[0:3] = mu.T
    P[3:6] = rng.normal(-2.6, 0.3, (3, n))
    P[6:10] = rng.normal(size=(4, n))
    P[10] = rng.normal(0.0, 1.0, n)
    P[11:14] = rng.uniform(-1.0, 1.0, (3, n))
    P[14:] = rng.normal(0.0, 0.2, (P.shape[0] - 14, n))
    return P, cam


@pytest.mark.parametrize("seed", [0, 1])
def test_gradients_match_central_differences(seed):
    P, cam = _fd_scene(seed)
    bg = np.array([0.3, 0.1, 0.2])
    rng = np.random.default_rng(50 + seed)
    wc = rng.normal(size=(3, 48, 64))
    wd = rng.normal(size=(48, 64)) * 0.1
    rec = osp.preprocess(P, 3, cam, requires_grad=True)
    img = osp.composite(rec, bg)
    # keep threshold decisions away from the finite-difference step
    bad = (img.margin_alpha < 1e-3) | (img.margin_T < 1e-3) | (img.margin_clamp < 1e-3)
    wc[:, bad] = 0.0
    wd[bad] = 0.0
    assert (~rec.culled).sum() > 30 and (rec.raw_rgb_margin > 1e-5).all()
    gr = osp.render_grad(rec, img, wc, wd)

    def objective(Pm):
        r, im = osp.render(Pm, 3, cam, bg)
        return float((im.rgb.detach().numpy() * wc).sum() + (im.depth.detach().numpy() * wd).sum())

    checked = 0
    for g in np.nonzero(~rec.culled)[0][:5]:
        for row in range(P.shape[0]):
            h = 1e-6 * max(1.0, abs(P[row, g]))
            Pp, Pm = P.copy(), P.copy()
            Pp[row, g] += h
            Pm[row, g] -= h
            fd = (objective(Pp) - objective(Pm)) / (2 * h)
            ad = gr.params[row, g]
            assert abs(fd - ad) <= 1e-7 + 1e-5 * abs(ad), (g, row, fd, ad)
            checked += 1
    assert checked == 5 * P.shape[0]


def test_l1_loss_and_psnr_hand_values():
    rgb = np.array([0.5, 0.25, 1.0, 0.0]).reshape(1, 2, 2)
    tgt = np.array([0.25, 0.25, 0.5, 0.5]).reshape(1, 2, 2)
    loss, g, _ = osp.l1_loss(rgb, tgt)
    assert loss == pytest.approx((0.25 + 0 + 0.5 + 0.5) / 4)
    assert g.ravel().tolist() == [0.25, 0.0, 0.25, -0.25]
    mse = (0.25 ** 2 + 0 + 0.5 ** 2 + 0.5 ** 2) / 4
    assert osp.psnr(rgb, tgt) == pytest.approx(10 * math.log10(1 / mse))
