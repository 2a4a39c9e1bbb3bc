"""Pins of the loss oracle (Eqs. 2-4): window, blur, SSIM special cases,
reductions, and finite-difference gradients."""
import numpy as np
import scipy.signal
import torch

from oracle import loss as ol


def test_window_is_normalised_gaussian():
    g = ol.gaussian_window().numpy()
    ref = scipy.signal.windows.gaussian(11, 1.5)
    assert np.allclose(g, ref / ref.sum(), atol=1e-15)
    assert abs(g.sum() - 1.0) < 1e-15


def test_blur_matches_brute_force():
    rng = np.random.default_rng(0)
    img = rng.uniform(size=(2, 9, 14))
    g = ol.gaussian_window().numpy()
    ref = np.zeros_like(img)
    for c in range(2):
        for i in range(9):
            for j in range(14):
                acc = 0.0
                for a in range(11):
                    for b in range(11):
                        ii, jj = i + a - 5, j + b - 5
                        if 0 <= ii < 9 and 0 <= jj < 14:
                            acc += g[a] * g[b] * img[c, ii, jj]
                ref[c, i, j] = acc
    got = ol.blur(torch.tensor(img)).numpy()
    assert np.abs(got - ref).max() < 1e-14


def test_ssim_special_cases():
    rng = np.random.default_rng(1)
    x = torch.tensor(rng.uniform(size=(3, 20, 24)))
    assert torch.equal(ol.ssim_map(x, x), torch.ones_like(x))
    a, b = 0.3, 0.7
    xa = torch.full((1, 30, 30), a, dtype=torch.float64)
    yb = torch.full((1, 30, 30), b, dtype=torch.float64)
    s = ol.ssim_map(xa, yb)
    # away from the border the window sees constants: variances vanish
    ref = (2 * a * b + ol.C1) / (a * a + b * b + ol.C1)
    assert abs(s[0, 15, 15].item() - ref) < 1e-12
    y = torch.tensor(rng.uniform(size=(3, 20, 24)))
    assert torch.allclose(ol.ssim_map(x, y), ol.ssim_map(y, x), atol=1e-15)
    assert (ol.ssim_map(x, y) < 1).all()


def test_loss_reduces_to_its_terms():
    rng = np.random.default_rng(2)
    x = rng.uniform(size=(2, 3, 16, 18))
    y = rng.uniform(size=(2, 3, 16, 18))
    d = rng.uniform(1, 5, size=(2, 16, 18))
    dt = rng.uniform(1, 5, size=(2, 16, 18))
    l1 = sum(np.abs(x[v] - y[v]).mean() for v in range(2))
    assert abs(ol.mapping_loss(x, y, lambda_s=0.0).item() - l1) < 1e-13
    s = sum(1 - ol.ssim_map(torch.tensor(x[v]), torch.tensor(y[v])).mean().item() for v in range(2))
    assert abs(ol.mapping_loss(x, y, lambda_s=1.0).item() - s) < 1e-13
    dl = sum(np.abs(d[v] - dt[v]).mean() for v in range(2))
    full = ol.mapping_loss(x, y, d, dt, lambda_s=0.2, lambda_depth=0.5).item()
    assert abs(full - (0.8 * l1 + 0.2 * s + 0.5 * dl)) < 1e-12


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    x = rng.uniform(size=(1, 3, 7, 9))
    y = rng.uniform(size=(1, 3, 7, 9))
    d = rng.uniform(1, 5, size=(1, 7, 9))
    dt = d + rng.choice([-1, 1], size=d.shape) * rng.uniform(0.1, 1, size=d.shape)
    L, gx, gd = ol.mapping_loss_grad(x, y, d, dt, lambda_s=0.3, lambda_depth=0.7)
    h = 1e-6
    for idx in [(0, 0, 0, 0), (0, 1, 3, 4), (0, 2, 6, 8), (0, 0, 3, 0), (0, 1, 0, 5)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (ol.mapping_loss(xp, y, d, dt, 0.3, 0.7).item() -
              ol.mapping_loss(xm, y, d, dt, 0.3, 0.7).item()) / (2 * h)
        assert abs(fd - gx[idx]) <= 1e-8 + 1e-6 * abs(gx[idx]), (idx, fd, gx[idx])
    for idx in [(0, 0, 0), (0, 3, 4), (0, 6, 8)]:
        dp, dm = d.copy(), d.copy()
        dp[idx] += h
        dm[idx] -= h
        fd = (ol.mapping_loss(x, y, dp, dt, 0.3, 0.7).item() -
              ol.mapping_loss(x, y, dm, dt, 0.3, 0.7).item()) / (2 * h)
        assert abs(fd - gd[idx]) <= 1e-8 + 1e-6 * abs(gd[idx])


def test_stability_constants_follow_the_ssim_definition():
    # C1 = (K1 L)^2, C2 = (K2 L)^2 with K1 = 0.01, K2 = 0.03 (Wang et al.,
    # 2004) and dynamic range L = 1 for colours in [0, 1]
    assert ol.C1 == (0.01 * 1.0) ** 2 and ol.C2 == (0.03 * 1.0) ** 2
    # C2 enters only where the window sees variance: a step edge
    x = torch.zeros((1, 21, 21), dtype=torch.float64)
    x[:, :, 11:] = 1.0
    y = torch.zeros_like(x)
    y[:, :, 10:] = 1.0
    s = ol.ssim_map(x, y)[0, 10, 10].item()
    mx, my = ol.blur(x), ol.blur(y)
    vx = (ol.blur(x * x) - mx * mx)[0, 10, 10].item()
    assert vx > 0.1 and 0.5 < s < 1.0
