"""Oracle: Gaussian projection, tile keys, compositing, loss and gradients.

TEST INFRASTRUCTURE ONLY (see the package header).

The paper's rasterizer renders RGB and depth of the visible Gaussians for a
keyframe and is optimised through the losses of Eqs. (2)-(4) (Sec. III-C and
Sec. III-E).  It fixes no formula of the splatting itself beyond citing
3D Gaussian Splatting, so the readings below define it; they are the ones the
HIP library implements.

Parameterisation (per Gaussian, raw values):
    scale s = exp(log_scale); opacity o = sigmoid(logit);
    q_hat = q/|q| (w, x, y, z) -> rotation R; Sigma = R S S^T R^T;
    colour = max(sum_k f_k Y_k(d) + 0.5, 0) per channel, d = unit vector from
    the camera centre to the mean (real SH basis of ``oracle.sh``).
Projection (pinhole, x right / y down / z forward, pixel (i, j) centred at
(i + 0.5, j + 0.5)):
    (X, Y, Z) = R_cw mu + t_cw;  u = fx X/Z + cx;  v = fy Y/Z + cy;
    J = [[fx/Z, 0, -fx X/Z^2], [0, fy/Z, -fy Y/Z^2]];
    Sigma2 = J R_cw Sigma R_cw^T J^T + 0.3 I;  conic Q = Sigma2^-1.
Culled (never drawn): Z <= z_near; |X/Z| > 1.3 (W/2)/fx; |Y/Z| > 1.3 (H/2)/fy;
    o < 1/255; det(Sigma2) <= 0; or an empty pixel box.
Pixel box: r^2 = 2 ln(255 o), e_x = sqrt(r^2 Sigma2_xx), e_y likewise; columns
    ceil(u - e_x - 0.5) .. floor(u + e_x - 0.5) clipped to the image, rows
    likewise.  Outside this box alpha < 1/255 exactly, so the image does not
    depend on the tile size.
Tiles: a drawn Gaussian is binned to every tile of the rectangle of tiles
    its pixel box touches (floor(i/TW), floor(j/TH) of the box corners).
Order: by the float32 rounding of Z (its bit pattern), then by index.
Compositing at pixel p, over the Gaussians whose box holds p, front to back:
    power = -1/2 d^T Q d with d = p - (u, v); skip if power > 0;
    alpha = min(0.99, o e^power); skip if alpha < 1/255;
    stop before a Gaussian that would take T below 1e-4;
    C += colour alpha T;  D += Z alpha T;  T *= 1 - alpha.
    Output C + T bg, D (no background depth), final T.
Loss: mean L1 over the 3HW colour values, optionally + lambda mean L1 on depth.
Gradients: reverse-mode derivative of the float64 forward above (torch
    autograd); thresholds and clamps pass no derivative.

Pins (tests/test_oracle_splat.py): the isotropic single Gaussian in closed
form, zero opacity giving the background exactly, two-Gaussian compositing,
the 13-deep stack at alpha = 1/2, the 0.99 clamp, the projection Jacobian
against finite differences of the projection, quaternion rotation against
Hamilton products, brute-force box containment of every alpha >= 1/255
sample, keys and ranges against a linear scan, the per-pair alpha maximum
against closed forms and per-pixel evaluation, and central finite
differences of the forward for every parameter row.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from .sh import sh_basis

F64 = torch.float64
GUARD = 1.3
DILATION = 0.3
ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99
T_MIN = 1e-4


def quat_to_rotmat(q: torch.Tensor) -> torch.Tensor:
    """Unit quaternions [n, 4] (w, x, y, z) -> rotation matrices [n, 3, 3]."""
    w, x, y, z = q.unbind(1)
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], 1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], 1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], 1),
    ], 1)


@dataclass
class Records:
    """Per-Gaussian projection of one view (float64; u..rgb carry autograd)."""
    params: torch.Tensor          # [R, n] leaf
    u: torch.Tensor
    v: torch.Tensor
    conic: torch.Tensor           # [n, 3]: Q00, Q01, Q11
    opacity: torch.Tensor
    rgb: torch.Tensor             # [n, 3]
    z: torch.Tensor
    zbits: np.ndarray             # int64 bit pattern of float32(Z)
    culled: np.ndarray            # bool
    box: np.ndarray               # int64 [n, 4]: i0, i1, j0, j1 (inclusive)
    tile_rect: np.ndarray         # int64 [n, 4]: tx0, tx1, ty0, ty1
    raw_rgb_margin: np.ndarray    # |colour before clamp| (gradient switch)
    key_tie: np.ndarray           # bool: some integer decision within 1e-13 of a flip
    width: int
    height: int
    tile: tuple


def preprocess(params: np.ndarray, sh_degree: int, cam: dict, tile=(16, 16),
               requires_grad: bool = False) -> Records:
    P = torch.tensor(np.asarray(params, np.float64), dtype=F64, requires_grad=requires_grad)
    n = P.shape[1]
    K = (sh_degree + 1) ** 2
    mean = P[0:3].T
    scale = torch.exp(P[3:6].T)
    quat = P[6:10].T
    opac = torch.sigmoid(P[10])
    sh = P[11:11 + 3 * K].reshape(K, 3, n)

    qn = quat / torch.linalg.norm(quat, dim=1, keepdim=True)
    Rg = quat_to_rotmat(qn)
    M = Rg * scale[:, None, :]
    Sigma = M @ M.transpose(1, 2)

    Rc = torch.tensor(cam["R"], dtype=F64)
    tc = torch.tensor(cam["t"], dtype=F64)
    fx, fy, cx, cy = cam["fx"], cam["fy"], cam["cx"], cam["cy"]
    W, H = cam["width"], cam["height"]
    Xc = mean @ Rc.T + tc
    X, Y, Z = Xc.unbind(1)
    zero = torch.zeros_like(Z)
    J = torch.stack([torch.stack([fx / Z, zero, -fx * X / (Z * Z)], 1),
                     torch.stack([zero, fy / Z, -fy * Y / (Z * Z)], 1)], 1)
    Sig_c = Rc @ Sigma @ Rc.T
    S2 = J @ Sig_c @ J.transpose(1, 2)
    a = S2[:, 0, 0] + DILATION
    b = S2[:, 0, 1]
    c = S2[:, 1, 1] + DILATION
    det = a * c - b * b
    conic = torch.stack([c / det, -b / det, a / det], 1)
    u = fx * X / Z + cx
    v = fy * Y / Z + cy

    centre = -(Rc.T @ tc)
    dvec = mean - centre
    dirs = dvec / torch.linalg.norm(dvec, dim=1, keepdim=True)
    basis = sh_basis(dirs, sh_degree)                      # [n, K]
    raw = torch.einsum("nk,kcn->nc", basis, sh) + 0.5
    rgb = torch.clamp(raw, min=0.0)

    with torch.no_grad():
        Zd, Xd, Yd = Z.numpy(), X.numpy(), Y.numpy()
        od, ad, cd, dd = opac.numpy(), a.numpy(), c.numpy(), det.numpy()
        ud, vd = u.numpy(), v.numpy()
        lim_x = GUARD * 0.5 * W / fx
        lim_y = GUARD * 0.5 * H / fy
        with np.errstate(divide="ignore", invalid="ignore"):
            rx = np.abs(Xd / Zd)
            ry = np.abs(Yd / Zd)
            culled = (Zd <= cam["z_near"]) | (rx > lim_x) | (ry > lim_y) | (od < ALPHA_MIN) | (dd <= 0)
            r2 = np.where(culled, 0.0, 2.0 * np.log(255.0 * od))
            ex = np.sqrt(r2 * np.where(culled, 0.0, ad))
            ey = np.sqrt(r2 * np.where(culled, 0.0, cd))
            e0, e1 = ud - ex - 0.5, ud + ex - 0.5
            f0, f1 = vd - ey - 0.5, vd + ey - 0.5
            big = 1e9
            i0 = np.maximum(np.ceil(np.clip(e0, -big, big)), 0)
            i1 = np.minimum(np.floor(np.clip(e1, -big, big)), W - 1)
            j0 = np.maximum(np.ceil(np.clip(f0, -big, big)), 0)
            j1 = np.minimum(np.floor(np.clip(f1, -big, big)), H - 1)
        culled = culled | (i0 > i1) | (j0 > j1) | ~np.isfinite(ud) | ~np.isfinite(vd)
        box = np.stack([i0, i1, j0, j1], 1)
        box = np.where(culled[:, None], 0, box).astype(np.int64)
        TW, TH = tile
        rect = np.stack([box[:, 0] // TW, box[:, 1] // TW, box[:, 2] // TH, box[:, 3] // TH], 1)
        zf = Zd.astype(np.float32)
        zbits = zf.view(np.int32).astype(np.int64)

        # Margins of every integer decision that is actually reached
        # (relative); 1e-13 is far above the float64 disagreement of two
        # correct implementations (~1e-15).
        def frac_margin(x):
            return np.abs(x - np.round(x)) / np.maximum(1.0, np.abs(x))
        inf = np.full(Zd.shape, np.inf)
        with np.errstate(divide="ignore", invalid="ignore"):
            front = Zd > cam["z_near"]
            m_near = np.abs(Zd - cam["z_near"]) / cam["z_near"]
            m_guard = np.where(front, np.minimum(np.abs(rx - lim_x) / lim_x, np.abs(ry - lim_y) / lim_y), inf)
            m_opac = np.abs(255.0 * od - 1.0)
            reach_box = front & (rx <= lim_x) & (ry <= lim_y) & (od >= ALPHA_MIN) & (dd > 0)
            m_box = np.where(reach_box, np.minimum.reduce([frac_margin(e0), frac_margin(e1),
                                                           frac_margin(f0), frac_margin(f1)]), inf)
            m = np.minimum.reduce([m_near, m_guard, m_opac, m_box])
            ulp = np.abs(np.nextafter(zf, np.float32(np.inf)).astype(np.float64) - zf.astype(np.float64))
            mz = np.where(culled, inf, np.abs(np.abs(Zd - zf.astype(np.float64)) - 0.5 * ulp) / np.abs(Zd))
        key_tie = (m < 1e-13) | (mz < 1e-13)
        rgb_margin = np.abs(raw.numpy()).min(axis=1)

    # The composited depth is its own graph node, so its gradient is the
    # depth-channel term alone (Z also reaches u, v and the conic).
    return Records(params=P, u=u, v=v, conic=conic, opacity=opac, rgb=rgb, z=Z.clone(), zbits=zbits,
                   culled=culled, box=box, tile_rect=rect, raw_rgb_margin=rgb_margin,
                   key_tie=key_tie, width=W, height=H, tile=tuple(tile))


def pair_alpha_max(rec: Records, g: np.ndarray, tx: np.ndarray, ty: np.ndarray) -> np.ndarray:
    """For (Gaussian g, tile (tx, ty)) pairs: the largest float64 alpha
    before the 0.99 clamp, o exp(-1/2 d^T Q d), over the pixel centres that
    lie both in the tile and in the Gaussian's pixel box (brute force over
    every such centre; -inf where the two share no pixel).  A pair whose
    value is below 1/255 adds nothing to any pixel of its tile."""
    TW, TH = rec.tile
    g = np.asarray(g, np.int64)
    tx = np.asarray(tx, np.int64)
    ty = np.asarray(ty, np.int64)
    u = rec.u.detach().numpy()[g]
    v = rec.v.detach().numpy()[g]
    Q = rec.conic.detach().numpy()[g]
    o = rec.opacity.detach().numpy()[g]
    box = rec.box[g]
    best = np.full(g.shape, -np.inf)
    for oy in range(TH):
        j = ty * TH + oy
        in_y = (j >= box[:, 2]) & (j <= box[:, 3])
        dy = j + 0.5 - v
        for ox in range(TW):
            i = tx * TW + ox
            ok = in_y & (i >= box[:, 0]) & (i <= box[:, 1])
            dx = i + 0.5 - u
            a = o * np.exp(-0.5 * (Q[:, 0] * dx * dx + 2.0 * Q[:, 1] * dx * dy + Q[:, 2] * dy * dy))
            best = np.where(ok, np.maximum(best, a), best)
    return best


def tile_keys(rec: Records, view: int = 0, tiles_before: int = 0) -> dict:
    """Keys (tile << 32 | float32 depth bits) and values (Gaussian index) for
    every (drawn Gaussian, tile of its rectangle), emitted by index then
    tiles row-major; then a stable sort and per-tile [start, end) ranges.
    `tiles_before` is the global tile id of this view's tile 0.  Also
    returns each pair's Gaussian and tile coordinates in sorted order."""
    TW, TH = rec.tile
    tx_n = -(-rec.width // TW)
    ty_n = -(-rec.height // TH)
    vis = np.nonzero(~rec.culled)[0]
    r = rec.tile_rect
    wcount = r[vis, 1] - r[vis, 0] + 1
    hcount = r[vis, 3] - r[vis, 2] + 1
    cnt = wcount * hcount
    g = np.repeat(vis, cnt)
    start = np.repeat(np.cumsum(cnt) - cnt, cnt)
    local = np.arange(cnt.sum()) - start
    wrep = np.repeat(wcount, cnt)
    tx = r[g, 0] + local % wrep
    ty = r[g, 2] + local // wrep
    tile_id = tiles_before + ty * tx_n + tx
    keys = (tile_id.astype(np.uint64) << np.uint64(32)) | rec.zbits[g].astype(np.uint64)
    vals = g.astype(np.int64)
    order = np.argsort(keys, kind="stable")
    ks, vs = keys[order], vals[order]
    t_of = (ks >> np.uint64(32)).astype(np.int64)
    all_t = np.arange(tiles_before, tiles_before + tx_n * ty_n)
    lo = np.searchsorted(t_of, all_t, "left")
    hi = np.searchsorted(t_of, all_t, "right")
    counts = np.zeros(rec.culled.size, np.int64)
    np.add.at(counts, g, 1)
    return dict(keys=ks, values=vs, ranges=np.stack([lo, hi], 1), counts=counts,
                tiles_x=tx_n, tiles_y=ty_n, tx=tx[order], ty=ty[order])


@dataclass
class Image:
    rgb: torch.Tensor        # [3, h, w]
    depth: torch.Tensor      # [h, w]
    T: torch.Tensor          # [h, w]
    n_contrib: np.ndarray    # [h, w] number of included Gaussians
    last_g: np.ndarray       # [h, w] index of the last included Gaussian, -1 if none
    margin_alpha: np.ndarray  # [h, w] min |alpha/(1/255) - 1| over the pixel's samples
    margin_T: np.ndarray      # [h, w] min |T_after/1e-4 - 1|
    margin_clamp: np.ndarray  # [h, w] min |o G / 0.99 - 1|
    crop: tuple


def composite(rec: Records, bg, crop=None) -> Image:
    """Per-pixel front-to-back compositing over the whole image or over the
    half-open pixel window crop = (x0, x1, y0, y1)."""
    W, H = rec.width, rec.height
    x0, x1, y0, y1 = crop if crop is not None else (0, W, 0, H)
    w, h = x1 - x0, y1 - y0
    vis = np.nonzero(~rec.culled)[0]
    bi0 = np.maximum(rec.box[vis, 0], x0)
    bi1 = np.minimum(rec.box[vis, 1], x1 - 1)
    bj0 = np.maximum(rec.box[vis, 2], y0)
    bj1 = np.minimum(rec.box[vis, 3], y1 - 1)
    bw = np.maximum(bi1 - bi0 + 1, 0)
    bh = np.maximum(bj1 - bj0 + 1, 0)
    area = bw * bh
    E = int(area.sum())
    g = np.repeat(vis, area)
    start = np.repeat(np.cumsum(area) - area, area)
    local = np.arange(E) - start
    wrep = np.repeat(bw, area)
    pi = np.repeat(bi0, area) + local % np.maximum(wrep, 1)
    pj = np.repeat(bj0, area) + local // np.maximum(wrep, 1)
    pix = (pj - y0) * w + (pi - x0)
    key = (pix.astype(np.int64) << 32) | rec.zbits[g]
    order = np.argsort(key, kind="stable")      # ties keep ascending Gaussian index
    g, pi, pj, pix = g[order], pi[order], pj[order], pix[order]

    gt = torch.from_numpy(g)
    dx = torch.from_numpy(pi + 0.5) - rec.u[gt]
    dy = torch.from_numpy(pj + 0.5) - rec.v[gt]
    Q = rec.conic[gt]
    power = -0.5 * (Q[:, 0] * dx * dx + Q[:, 2] * dy * dy) - Q[:, 1] * dx * dy
    oG = rec.opacity[gt] * torch.exp(power)
    alpha = torch.clamp(oG, max=ALPHA_MAX)
    skip = (power > 0) | (alpha < ALPHA_MIN)

    npix = w * h
    pixt = torch.from_numpy(pix)
    counts = np.bincount(pix, minlength=npix)
    seg_start = np.repeat(np.cumsum(counts) - counts, counts)
    seg_start_t = torch.from_numpy(seg_start)

    def seg_cumsum(x):
        cs = torch.cumsum(x, 0)
        if x.numel() == 0:
            return cs
        base = (cs - x)[seg_start_t]
        return cs - base

    with torch.no_grad():
        a_eff = torch.where(skip, torch.zeros_like(alpha), alpha)
        T_after = torch.exp(seg_cumsum(torch.log1p(-a_eff)))
        included = (~skip) & (T_after >= T_MIN)
    a_inc = torch.where(included, alpha, torch.zeros_like(alpha))
    la = torch.log1p(-a_inc)
    T_before = torch.exp(seg_cumsum(la) - la)
    wgt = a_inc * T_before
    C = torch.zeros(npix, 3, dtype=F64).index_add(0, pixt, rec.rgb[gt] * wgt[:, None])
    D = torch.zeros(npix, dtype=F64).index_add(0, pixt, rec.z[gt] * wgt)
    T = torch.exp(torch.zeros(npix, dtype=F64).index_add(0, pixt, la))
    bg_t = torch.tensor(np.asarray(bg, np.float64), dtype=F64)
    C_out = C + T[:, None] * bg_t[None, :]

    with torch.no_grad():
        inc = included.numpy()
        n_contrib = np.bincount(pix[inc], minlength=npix)
        last_pos = np.full(npix, -1, np.int64)
        np.maximum.at(last_pos, pix[inc], np.nonzero(inc)[0])
        last_g = np.where(last_pos >= 0, g[np.maximum(last_pos, 0)] if E else -1, -1)
        big = np.inf
        al = oG.numpy()
        ok = ~(power.numpy() > 0)
        m_a = np.where(ok, np.abs(al / ALPHA_MIN - 1.0), big)
        m_t = np.where(~skip.numpy(), np.abs(T_after.numpy() / T_MIN - 1.0), big)
        m_c = np.where(ok, np.abs(al / ALPHA_MAX - 1.0), big)

        def seg_min(x):
            out = np.full(npix, big)
            np.minimum.at(out, pix, x)
            return out
        margin_alpha, margin_T, margin_clamp = seg_min(m_a), seg_min(m_t), seg_min(m_c)

    return Image(rgb=C_out.T.reshape(3, h, w), depth=D.reshape(h, w), T=T.reshape(h, w),
                 n_contrib=n_contrib.reshape(h, w), last_g=last_g.reshape(h, w),
                 margin_alpha=margin_alpha.reshape(h, w), margin_T=margin_T.reshape(h, w),
                 margin_clamp=margin_clamp.reshape(h, w), crop=(x0, x1, y0, y1))


@dataclass
class Gradients:
    params: np.ndarray       # [R, n] d(objective)/d(raw parameter)
    uv: np.ndarray           # [n, 2]
    conic: np.ndarray        # [n, 3]
    opacity: np.ndarray      # [n]   (w.r.t. the activated opacity o)
    rgb: np.ndarray          # [n, 3]
    z: np.ndarray            # [n]


def render_grad(rec: Records, img: Image, dl_drgb, dl_ddepth=None) -> Gradients:
    """Gradient of sum(dl_drgb * rgb) + sum(dl_ddepth * depth) over the image
    (or crop) that `img` holds, i.e. the vector-Jacobian product with the
    given upstream gradients.  `rec` must come from preprocess(...,
    requires_grad=True)."""
    for t in (rec.u, rec.v, rec.conic, rec.opacity, rec.rgb, rec.z):
        t.retain_grad()
    obj = (img.rgb * torch.tensor(np.asarray(dl_drgb, np.float64))).sum()
    if dl_ddepth is not None:
        obj = obj + (img.depth * torch.tensor(np.asarray(dl_ddepth, np.float64))).sum()
    obj.backward()

    def g(t, shape):
        return t.grad.numpy().copy() if t.grad is not None else np.zeros(shape)
    n = rec.params.shape[1]
    return Gradients(params=g(rec.params, tuple(rec.params.shape)),
                     uv=np.stack([g(rec.u, (n,)), g(rec.v, (n,))], 1),
                     conic=g(rec.conic, (n, 3)), opacity=g(rec.opacity, (n,)),
                     rgb=g(rec.rgb, (n, 3)), z=g(rec.z, (n,)))


def l1_loss(rgb, target, depth=None, depth_target=None, lambda_depth: float = 0.0):
    """Eqs. (2)-(4) without the SSIM term: mean |C - C_gt| over the 3HW colour
    values, plus lambda_depth * mean |D - D_gt| when a depth target is given.
    Returns (loss, dL/dC, dL/dD or None); sign(0) = 0."""
    rgb = np.asarray(rgb, np.float64)
    target = np.asarray(target, np.float64)
    diff = rgb - target
    loss = np.abs(diff).mean()
    g = np.sign(diff) / diff.size
    gd = None
    if depth_target is not None and lambda_depth != 0.0:
        dd = np.asarray(depth, np.float64) - np.asarray(depth_target, np.float64)
        loss += lambda_depth * np.abs(dd).mean()
        gd = lambda_depth * np.sign(dd) / dd.size
    return loss, g, gd


def psnr(rgb, target) -> float:
    """10 log10(1 / MSE) over 3HW values, rendered colour clipped to [0, 1]."""
    mse = np.mean((np.clip(np.asarray(rgb, np.float64), 0, 1) - np.asarray(target, np.float64)) ** 2)
    return float(10.0 * math.log10(1.0 / mse))


def render(params, sh_degree, cam, bg, tile=(16, 16), crop=None):
    """Convenience: preprocess + composite without gradients."""
    rec = preprocess(params, sh_degree, cam, tile)
    return rec, composite(rec, bg, crop)
