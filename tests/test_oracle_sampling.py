"""Pins of the LoG sampling oracle."""
import numpy as np

from oracle import sampling as osm


def test_second_derivative_kernel_is_the_analytic_derivative():
    g, d2 = osm.log_kernels(1.0)
    x = np.arange(-4, 5, dtype=np.float64)
    # d^2/dx^2 of c exp(-x^2 / 2) is c (x^2 - 1) exp(-x^2 / 2)
    assert np.allclose(d2, (x * x - 1.0) * g, atol=1e-16)
    assert abs(g.sum() - 1.0) < 1e-15 and np.allclose(g, g[::-1])
    # applied to a constant the second-derivative filter gives sum(d2)
    assert abs(np.sum(d2 * 3.0) - 3.0 * d2.sum()) < 1e-15


def _reflect(i, n):
    # mirror with the edge sample repeated: -1 -> 0, n -> n - 1
    while i < 0 or i >= n:
        i = -i - 1 if i < 0 else 2 * n - 1 - i
    return i


def test_log_response_matches_brute_force_convolution():
    rng = np.random.default_rng(0)
    img = rng.uniform(size=(3, 11, 13))
    g, d2 = osm.log_kernels(1.0)
    r = len(g) // 2
    ref = np.zeros((3, 11, 13))
    for c in range(3):
        for i in range(11):
            for j in range(13):
                acc = 0.0
                for a in range(-r, r + 1):
                    for b in range(-r, r + 1):
                        v = img[c, _reflect(i + a, 11), _reflect(j + b, 13)]
                        acc += (d2[a + r] * g[b + r] + g[a + r] * d2[b + r]) * v
                ref[c, i, j] = acc
    got = osm.log_response(img)
    assert np.abs(got - np.sqrt((ref ** 2).sum(0))).max() < 1e-12


def test_linear_image_response_in_closed_form():
    # symmetric kernels kill the odd moments, so inside the image the LoG of
    # a + b x + c y is 2 (sum d2) (a + b x + c y): the truncated
    # second-derivative kernel does not sum to zero
    g, d2 = osm.log_kernels(1.0)
    yy, xx = np.mgrid[0:20, 0:24].astype(np.float64)
    img = np.stack([0.01 * xx, 0.02 * yy, 0.5 + 0.0 * xx])
    resp = osm.log_response(img)
    ref = np.abs(2.0 * d2.sum()) * np.sqrt((img ** 2).sum(0))
    assert np.abs(resp - ref)[5:-5, 5:-5].max() < 1e-15


def test_sampling_map_special_cases_and_selection():
    rng = np.random.default_rng(1)
    img = rng.uniform(size=(3, 16, 20))
    assert (osm.sampling_map(img, img) == 0).all()
    flat = np.zeros_like(img)          # no LoG response at all
    ps = osm.sampling_map(img, flat)
    assert np.allclose(ps, np.minimum(1.0, 2.0 * osm.log_response(img)))
    u = rng.uniform(size=(16, 20))
    sel, ties = osm.sample_pixels(img, flat, u)
    brute = [y * 20 + x for y in range(16) for x in range(20) if u[y, x] < ps[y, x]]
    assert list(sel) == brute and len(brute) > 0
    assert ties.sum() <= 2


def test_detail_only_in_the_render_is_not_sampled():
    rng = np.random.default_rng(2)
    render = rng.uniform(size=(3, 12, 12))
    assert (osm.sampling_map(np.zeros_like(render), render) == 0).all()
