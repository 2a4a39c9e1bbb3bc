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
