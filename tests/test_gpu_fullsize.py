"""Parity at the headline workload's real size, in the launch configuration
bench.py times (indoor room, 5.75M Gaussians, ~2M active, 1200x680, 16x16
tiles): every tile key and range bit-exact; colour, depth and transmittance
on three sampled 64x64 crops; gradients of every Gaussian whose pixel box
lies inside the central crop (its whole gradient comes from that crop)."""
import numpy as np
import pytest
import torch

from gpu_helpers import IMG_TOL, assert_grad_close, check_pruned_keys, flagged_pixels
from oracle import chunks as oc
from oracle import splat as osp
from paper_2511_23030_amd import dcgs as D
from paper_2511_23030_amd import mapping

pytestmark = pytest.mark.gpu


def test_headline_keyframe(ctx):
    import bench
    w = bench.make_workload("indoor-2m")
    cam = w["cams"][3]
    W, H, deg, s = w["W"], w["H"], w["deg"], w["chunk"]
    print("case fullsize: workload generated", flush=True)
    pool = D.Pool(ctx, deg, budget=w["n"] + 1)
    pool.ingest(w["start"], s)
    loop = mapping.MappingLoop(ctx, pool, deg, s, 3_000_000, W, H, (16, 16))
    ids = loop.select(cam)
    # the oracle's own selection and compaction
    cid = oc.encode_id(oc.chunk_coord(w["start"][0:3].T, s))
    all_ids = np.unique(cid)
    ref_sel = oc.select_chunks([cam], all_ids, s)
    assert not ref_sel["tie"].any()
    assert (ids == ref_sel["union_ids"]).all()
    pool.require(ids, now=0)
    n = pool.compact(ids, loop.params, loop.src)
    order = np.argsort(cid, kind="stable")
    act = order[np.isin(cid[order], ids)]
    Pa = w["start"][:, act]
    assert n == Pa.shape[1] and 1.5e6 < n < 2.6e6
    assert (loop.params[:, :n].cpu().numpy() == Pa).all()
    print(f"case fullsize: {n} active", flush=True)

    bg = (0.0, 0.0, 0.0)
    T = torch.empty(H, W, device="cuda")
    loop.state.forward(loop.params, n, deg, cam, bg, (16, 16), loop.rgb, loop.depth, T)
    ex = loop.state.export(loop.params.device, H, W)
    rec = osp.preprocess(Pa, deg, cam, (16, 16), requires_grad=True)
    kr = osp.tile_keys(rec)
    tie = rec.key_tie
    assert tie.sum() < 1e-4 * n
    dropped, whole = check_pruned_keys(ex["keys"].cpu().numpy(), ex["values"].cpu().numpy(),
                                       ex["ranges"].cpu().numpy(), ex["counts"].cpu().numpy(),
                                       rec, kr, tie=tie, what="indoor keyframe")
    print(f"  {kr['keys'].size} oracle pairs, {dropped} left out as empty, {whole} Gaussians "
          f"left with no tile, {tie.sum()} key ties", flush=True)
    print("case fullsize: keys and ranges", flush=True)

    rgb, depth, Tg = loop.rgb.cpu().numpy(), loop.depth.cpu().numpy(), T.cpu().numpy()
    crops = [(568, 632, 308, 372), (0, 64, 0, 64), (1136, 1200, 616, 680)]
    rng = np.random.default_rng(9)
    dl = (rng.normal(size=(3, H, W)) * 1e-6).astype(np.float32)
    for k, (x0, x1, y0, y1) in enumerate(crops):
        img = osp.composite(rec, np.zeros(3), (x0, x1, y0, y1))
        flag = flagged_pixels(img)
        assert flag.sum() <= 0.05 * flag.size   # ~1000 candidates per pixel at this density
        ok = ~flag
        assert np.abs(rgb[:, y0:y1, x0:x1] - img.rgb.detach().numpy())[:, ok].max() <= IMG_TOL
        assert np.abs(Tg[y0:y1, x0:x1] - img.T.detach().numpy())[ok].max() <= IMG_TOL
        Dr = img.depth.detach().numpy()
        assert (np.abs(depth[y0:y1, x0:x1] - Dr)[ok] <= IMG_TOL * np.maximum(1, np.abs(Dr[ok]))).all()
        if k == 0:
            dl[:, y0:y1, x0:x1][:, flag] = 0.0
            central = (img, (x0, x1, y0, y1))
    print("case fullsize: images", flush=True)

    img, (x0, x1, y0, y1) = central
    box = rec.box
    inside = (~rec.culled & (box[:, 0] >= x0) & (box[:, 1] < x1) & (box[:, 2] >= y0)
              & (box[:, 3] < y1) & (rec.raw_rgb_margin > 1e-5))
    assert inside.sum() >= 50
    g_ref = osp.render_grad(rec, img, dl[:, y0:y1, x0:x1])
    grad = loop.state.backward(loop.params, n, torch.from_numpy(dl).cuda(), None, loop.grad)
    G = grad[:, :n].cpu().numpy()
    assert_grad_close(G[:, inside], g_ref.params[:, inside], "full-size gradients")
    pool.close()


def test_headline_window_in_the_bench_launch_configuration(ctx):
    """The bench's timed unit at full size: a 16-keyframe window rendered
    and differentiated in one launch sequence at the raster shape the
    autotuner picks for it (16x16 tiles, 4 pixels per lane forward and
    backward).  Every view's image and the summed gradient equal the
    per-view path bit for bit; one view's central crop against the oracle."""
    import bench
    w = bench.make_workload("indoor-2m")
    V = 16
    cams = w["cams"][:V]
    W, H, deg, s = w["W"], w["H"], w["deg"], w["chunk"]
    pool = D.Pool(ctx, deg, budget=w["n"] + 1)
    pool.ingest(w["start"], s)
    loop = mapping.MappingLoop(ctx, pool, deg, s, 3_400_000, W, H, (16, 16))
    loop._window_buffers(V)
    ids, masks = loop.select_window(cams)
    pool.require(ids, now=0)
    n = pool.compact(ids, loop.params, loop.src, masks=masks, out_gmask=loop.gmask)
    assert 2.0e6 < n < 3.4e6
    tile, ppt = (16, 16), 4 | 4 << 4
    print(f"case fullsize window: V={V} n={n}", flush=True)
    bg = (0.0, 0.0, 0.0)
    st_b = D.RenderState(ctx)
    rgb_b, depth_b = st_b.forward(loop.params, n, deg, cams, bg, tile, ppt=ppt, gmask=loop.gmask)
    rng = np.random.default_rng(8)
    dl = torch.from_numpy((rng.normal(size=(V, 3, H, W)) * 1e-7).astype(np.float32)).cuda()
    grad_b = st_b.backward(loop.params, n, dl, None)
    st_s = D.RenderState(ctx)
    grad_s = torch.empty_like(grad_b)
    for v in range(V):
        rgb, depth = st_s.forward(loop.params, n, deg, cams[v], bg, tile, ppt=ppt,
                                  gmask=loop.gmask, mask_shift=v)
        assert torch.equal(rgb, rgb_b[v]) and torch.equal(depth, depth_b[v]), v
        st_s.backward(loop.params, n, dl[v].contiguous(), None, grad_s, accumulate=v > 0)
    torch.cuda.synchronize()
    assert torch.equal(grad_b[:, :n], grad_s[:, :n])
    print("case fullsize window: batched equals per-view", flush=True)
    # view 5 of the window against the oracle on the central crop
    v = 5
    gm = loop.gmask[:n].cpu().numpy().astype(np.int64)
    Pv = loop.params[:, :n].cpu().numpy()[:, ((gm >> v) & 1) == 1]
    rec = osp.preprocess(Pv, deg, cams[v], (16, 16))
    x0, x1, y0, y1 = W // 2 - 32, W // 2 + 32, H // 2 - 32, H // 2 + 32
    img = osp.composite(rec, np.zeros(3), (x0, x1, y0, y1))
    flag = flagged_pixels(img)
    assert flag.sum() <= 0.05 * flag.size
    ok = ~flag
    got = rgb_b[v].cpu().numpy()[:, y0:y1, x0:x1]
    assert np.abs(got - img.rgb.detach().numpy())[:, ok].max() <= IMG_TOL
    pool.close()


def test_cell_skipping_changes_no_pixel_at_full_size(ctx):
    """The rasterizers skip 8x8 cells that a record's box or alpha >= 1/255
    ellipse misses.  Every raster shape composites each pixel with the same
    roundings, so a 16-keyframe window rendered with multi-cell tiles must
    equal, bit for bit, the same window with 8x8 tiles (one cell per tile,
    no cell masks): a cell skipped wrongly would change some pixel."""
    import bench
    w = bench.make_workload("indoor-2m")
    V = 16
    cams = w["cams"][8:8 + V]
    W, H, deg, s = w["W"], w["H"], w["deg"], w["chunk"]
    pool = D.Pool(ctx, deg, budget=w["n"] + 1)
    pool.ingest(w["start"], s)
    loop = mapping.MappingLoop(ctx, pool, deg, s, 3_400_000, W, H, (16, 16))
    loop._window_buffers(V)
    ids, masks = loop.select_window(cams)
    pool.require(ids, now=0)
    n = pool.compact(ids, loop.params, loop.src, masks=masks, out_gmask=loop.gmask)
    bg = (0.05, 0.1, 0.2)
    st = D.RenderState(ctx)
    T0 = torch.empty(V, H, W, device="cuda")
    rgb0, depth0 = st.forward(loop.params, n, deg, cams, bg, (8, 8), ppt=1, gmask=loop.gmask, T=T0)
    rgb0, depth0 = rgb0.clone(), depth0.clone()
    for tile, ppt in (((16, 16), 4), ((16, 16), 2), ((32, 16), 8)):
        print(f"case cell skipping: V={V} n={n} tile={tile} ppt={ppt}", flush=True)
        T1 = torch.empty(V, H, W, device="cuda")
        rgb1, depth1 = st.forward(loop.params, n, deg, cams, bg, tile, ppt=ppt, gmask=loop.gmask,
                                  T=T1)
        torch.cuda.synchronize()
        assert torch.equal(rgb1, rgb0) and torch.equal(depth1, depth0) and torch.equal(T1, T0)
    pool.close()
