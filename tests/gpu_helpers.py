"""Helpers shared by the GPU parity tests: run the HIP path through the C
ABI and compare with the oracle at the stated tolerances."""
import numpy as np
import torch

from paper_2511_23030_amd import dcgs as D

IMG_TOL = 1e-5          # max-abs on colour and transmittance (FP32 images)
GRAD_TOL = 1e-3         # relative, floor tau = 1e-3 * max |g_ref| per row
MARGIN_ALPHA = 1e-5     # relative margins below which a pixel's threshold
MARGIN_T = 1e-4         # decision may differ between FP32 and FP64
MARGIN_CLAMP = 1e-5


SHAPES = [(16, 16, 1), (16, 16, 2), (16, 16, 4), (8, 8, 1), (32, 16, 2), (32, 16, 4), (32, 16, 8)]


def gpu_render(ctx, params, deg, cam, bg, tile=(16, 16), dl=None, dld=None, ppt=0):
    H, W = cam["height"], cam["width"]
    Pt = torch.from_numpy(np.ascontiguousarray(params, np.float32)).cuda()
    n = Pt.shape[1]
    st = D.RenderState(ctx)
    T = torch.empty(H, W, dtype=torch.float32, device="cuda")
    rgb, depth = st.forward(Pt, n, deg, cam, bg, tile, T=T, ppt=ppt)
    ex = st.export(Pt.device, H, W)
    out = dict(rgb=rgb.cpu().numpy(), depth=depth.cpu().numpy(), T=T.cpu().numpy(),
               **{k: v.cpu().numpy() for k, v in ex.items()}, n_pairs=st.info()["n_pairs"])
    if dl is not None:
        g2d = torch.empty(10, max(n, 1), dtype=torch.float32, device="cuda")
        dl_t = torch.from_numpy(np.ascontiguousarray(dl, np.float32)).cuda()
        dld_t = None if dld is None else torch.from_numpy(np.ascontiguousarray(dld, np.float32)).cuda()
        grad = st.backward(Pt, n, dl_t, dld_t, grad2d=g2d)
        out["grad"] = grad.cpu().numpy()[:, :n]
        out["grad2d"] = g2d.cpu().numpy()[:, :n]
    torch.cuda.synchronize()
    st.close()
    return out


def flagged_pixels(img):
    return ((img.margin_alpha < MARGIN_ALPHA) | (img.margin_T < MARGIN_T)
            | (img.margin_clamp < MARGIN_CLAMP))


def assert_grad_close(g, ref, what, mask=None):
    """Elementwise |g - ref| <= GRAD_TOL * max(|ref|, tau) per row."""
    g = np.asarray(g, np.float64)
    ref = np.asarray(ref, np.float64)
    if mask is not None:
        g, ref = g[..., mask], ref[..., mask]
    if ref.size == 0:
        return
    tau = GRAD_TOL * np.abs(ref).max(axis=-1, keepdims=True)
    bound = GRAD_TOL * np.maximum(np.abs(ref), tau) + 1e-30
    bad = np.abs(g - ref) > bound
    if bad.any():
        idx = np.argwhere(bad)[:5]
        raise AssertionError(f"{what}: {bad.sum()} of {bad.size} entries off; first {idx.tolist()} "
                             f"gpu={g[tuple(idx.T)]} ref={ref[tuple(idx.T)]}")


def check_pruned_keys(gk, gv, granges, gcounts, rec, kr, tiles_before=0, tie=None, what=""):
    """The kernel's sorted (key, value) list against the oracle's plain list
    (every tile of each drawn Gaussian's rectangle).  The kernel may leave
    out (Gaussian, tile) pairs it has shown to hold no sample; the check:
      - the kernel list equals the oracle list with the left-out pairs
        removed, bit for bit and in the same order;
      - every left-out pair, including those of a Gaussian left with no tile
        at all, holds no pixel centre with alpha >= 1/255 (float64, brute
        force over the tile's pixels in the box);
      - per-tile ranges equal those of the oracle's list without the
        left-out pairs, and per-Gaussian counts its pair counts.
    Tiles touched by a Gaussian whose key sits within rounding of a decision
    (`tie`) are left out of the comparison.  Returns (pairs left out,
    Gaussians left with no tile)."""
    from oracle import splat as osp
    gk = np.asarray(gk).view(np.uint64)
    gv = np.asarray(gv).astype(np.int64)
    NT = kr["ranges"].shape[0]
    tb = np.uint64(tiles_before)
    t_o = ((kr["keys"] >> np.uint64(32)) - tb).astype(np.int64)
    t_k = ((gk >> np.uint64(32)) - tb).astype(np.int64)
    assert ((t_k >= 0) & (t_k < NT)).all(), what
    bad = np.zeros(NT, bool)
    tie = np.zeros(rec.culled.size, bool) if tie is None else tie
    for gi in np.nonzero(tie & ~rec.culled)[0]:
        t = rec.tile_rect[gi]
        for ty in range(t[2], t[3] + 1):
            bad[ty * kr["tiles_x"] + t[0]: ty * kr["tiles_x"] + t[1] + 1] = True
    id_o = kr["values"] * NT + t_o
    id_k = gv * NT + t_k
    kept = np.isin(id_o, id_k)
    ok_o, ok_k = ~bad[t_o], ~bad[t_k]
    assert np.array_equal(gk[ok_k], kr["keys"][kept & ok_o]), f"{what}: keys differ"
    assert np.array_equal(gv[ok_k], kr["values"][kept & ok_o]), f"{what}: values differ"
    assert np.isin(id_k[ok_k], id_o).all(), f"{what}: pair outside the oracle's list"
    drop = ~kept & ok_o
    if drop.any():
        amax = osp.pair_alpha_max(rec, kr["values"][drop], kr["tx"][drop], kr["ty"][drop])
        assert (amax < 1.0 / 255.0).all(), (
            f"{what}: {(amax >= 1 / 255).sum()} left-out pairs hold a sample, largest alpha {amax.max()}")
    g_lo = np.asarray(granges)[:, 0].astype(np.int64)
    g_hi = np.asarray(granges)[:, 1].astype(np.int64)
    all_t = np.arange(NT)
    if not bad.any():
        t_kept = t_o[kept]
        assert (g_lo == np.searchsorted(t_kept, all_t, "left")).all(), f"{what}: range starts"
        assert (g_hi == np.searchsorted(t_kept, all_t, "right")).all(), f"{what}: range ends"
    else:
        n_kept = np.bincount(t_o[kept], minlength=NT)
        assert ((g_hi - g_lo)[~bad] == n_kept[~bad]).all(), f"{what}: range lengths"
        assert (g_lo == np.searchsorted(t_k, all_t, "left")).all()
        assert (g_hi == np.searchsorted(t_k, all_t, "right")).all()
    n = rec.culled.size
    cnt = np.bincount(kr["values"][kept], minlength=n)
    ng = ~tie
    assert (np.asarray(gcounts)[:n][ng] == cnt[ng]).all(), f"{what}: per-Gaussian counts"
    whole = ~rec.culled & (kr["counts"] > 0) & (cnt == 0) & ng
    return int(drop.sum()), int(whole.sum())
