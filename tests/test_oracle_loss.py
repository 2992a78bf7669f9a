"""Pins of the mask and full-loss oracle (Sec. III-C, Eq. 7, 9-12) against what does not come
from the oracle itself: scipy's binary erosion and Gaussian filter, the SSIM closed form for an
affine pair of images, the maximum S = 1 at identical images, finite differences of the loss,
and invariance to pixels outside the mask."""
import numpy as np
import pytest
import scipy.ndimage as nd

import oracle
from oracle import loss_oracle as lo


def _disk(r):
    y, x = np.mgrid[-r:r + 1, -r:r + 1]
    return (x * x + y * y) <= r * r


@pytest.mark.parametrize("r", [0, 1, 2, 3, 5])
def test_erosion_matches_scipy(r):
    rng = np.random.default_rng(r)
    T = rng.random((37, 53)).astype(np.float32)
    # blobs, so the erosion keeps something
    T = nd.uniform_filter(T, 5).astype(np.float32)
    geo, inner = lo.support_masks(T, 0.5, r)
    assert np.array_equal(geo, T <= np.float32(0.5))
    exp = nd.binary_erosion(geo, structure=_disk(r), border_value=0) if r > 0 else geo
    assert np.array_equal(inner, exp)


def test_threshold_is_taken_in_float32():
    tau = 0.3
    thr = np.float32(1.0) - np.float32(tau)
    T = np.array([[np.nextafter(thr, np.float32(0)), thr, np.nextafter(thr, np.float32(2))]], np.float32)
    geo, _ = lo.support_masks(T, tau, 0)
    assert geo.tolist() == [[True, True, False]]


def test_window_matches_scipy_gaussian_filter():
    w = lo.gaussian_window()
    assert w.shape == (11, 11) and abs(w.sum() - 1.0) < 1e-15
    imp = np.zeros((11, 11))
    imp[5, 5] = 1.0
    np.testing.assert_allclose(nd.gaussian_filter(imp, 1.5, truncate=3.5, mode="constant"), w, rtol=1e-12,
                               atol=1e-15)
    rng = np.random.default_rng(1)
    img = rng.random((23, 31))
    np.testing.assert_allclose(lo.window_mean(img, w), nd.gaussian_filter(img, 1.5, truncate=3.5, mode="constant"),
                               rtol=1e-12, atol=1e-14)
    # the adjoint is the transpose of the linear map
    g = rng.standard_normal((23, 31))
    assert abs((lo.window_mean(img, w) * g).sum() - (img * lo.window_mean_adjoint(g, w)).sum()) < 1e-11


@pytest.mark.parametrize("a,b", [(1.0, 0.0), (0.7, 0.1), (-0.5, 0.6), (1.3, -0.2)])
def test_ssim_map_affine_closed_form(a, b):
    """Y = a X + b: mu_y = a mu_x + b, var_y = a^2 var_x, cov = a var_x inside the image."""
    rng = np.random.default_rng(2)
    X = nd.gaussian_filter(rng.random((40, 44)), 1.0)
    Y = a * X + b
    S = lo.ssim_terms(X, Y)["S"]
    f = lambda z: nd.gaussian_filter(z, 1.5, truncate=3.5, mode="constant")
    mx, vx = f(X), f(X * X) - f(X) ** 2
    my = a * mx + b
    exp = ((2 * mx * my + lo.SSIM_C1) / (mx * mx + my * my + lo.SSIM_C1)
           * (2 * a * vx + lo.SSIM_C2) / ((1 + a * a) * vx + lo.SSIM_C2))
    inner = (slice(5, -5), slice(5, -5))
    np.testing.assert_allclose(S[inner], exp[inner], rtol=1e-10, atol=1e-12)


def _images(seed, H=26, W=30):
    rng = np.random.default_rng(seed)
    rgb = nd.gaussian_filter(rng.random((3, H, W)), (0, 1.2, 1.2))
    tgt = np.clip(rgb + 0.15 * rng.standard_normal((3, H, W)), 0, 1)
    T = nd.uniform_filter(rng.random((H, W)), 7).astype(np.float32)
    _, M = lo.support_masks(T, 1.0 - float(np.median(T)), 1)
    return rng, rgb, tgt, M


def test_identical_images_are_the_maximum():
    rng, rgb, _, M = _images(3)
    L, g = lo.ssim_loss(rgb, rgb, M)
    assert abs(L) < 1e-12 and np.abs(g).max() < 1e-12
    L2, _ = lo.ssim_loss(rgb, rgb + 0.01 * rng.standard_normal(rgb.shape), M)
    assert L2 > 0


def test_ssim_gradient_matches_finite_differences():
    rng, rgb, tgt, M = _images(4)
    assert 0 < M.sum() < M.size
    L, g = lo.ssim_loss(rgb, tgt, M)
    h = 1e-6
    ys, xs = np.nonzero(M)
    pick = list(rng.choice(len(ys), 12, replace=False))
    pts = [(int(rng.integers(3)), int(ys[k]), int(xs[k])) for k in pick]
    pts += [(0, 0, 0), (2, M.shape[0] - 1, 3)]  # outside the mask: zero gradient
    for c, y, x in pts:
        p, m = rgb.copy(), rgb.copy()
        p[c, y, x] += h
        m[c, y, x] -= h
        fd = (lo.ssim_loss(p, tgt, M, want_grad=False)[0] - lo.ssim_loss(m, tgt, M, want_grad=False)[0]) / (2 * h)
        assert abs(fd - g[c, y, x]) <= 1e-6 * abs(g[c, y, x]) + 1e-9, (c, y, x, fd, g[c, y, x])


def test_pixels_outside_the_mask_do_not_matter():
    rng, rgb, tgt, M = _images(5)
    d = rng.standard_normal((26, 30))
    depth, tdepth = 3 + d, 3 + d + 0.1 * rng.standard_normal(d.shape)
    L, gC, gD = lo.masked_loss(rgb, depth, tgt, tdepth, M, 0.8, 0.2, 0.2)
    rgb2, depth2 = rgb.copy(), depth.copy()
    rgb2[:, ~M] = rng.random((3, int((~M).sum())))
    depth2[~M] += 5.0
    L2, gC2, gD2 = lo.masked_loss(rgb2, depth2, tgt, tdepth, M, 0.8, 0.2, 0.2)
    assert L == L2
    np.testing.assert_array_equal(gC, gC2)
    np.testing.assert_array_equal(gD, gD2)
    assert np.all(gC[:, ~M] == 0) and np.all(gD[~M] == 0)
    # restriction, not multiplication: non-finite values off the mask do not leak in
    rgb2[:, ~M] = np.nan
    depth2[~M] = np.inf
    L3, gC3, gD3 = lo.masked_loss(rgb2, depth2, tgt, tdepth, M, 0.8, 0.2, 0.2)
    assert L3 == L
    np.testing.assert_array_equal(gC3, gC)
    np.testing.assert_array_equal(gD3, gD)


def test_all_ones_mask_reduces_to_plain_l1_and_empty_mask_to_zero():
    rng, rgb, tgt, _ = _images(6)
    depth, tdepth = rng.random((26, 30)), rng.random((26, 30))
    L, gC, gD = lo.masked_loss(rgb, depth, tgt, tdepth, None, 1.0, 0.0, 0.2)
    L0, gC0, gD0 = oracle.l1_loss(rgb, depth, tgt, tdepth, 0.2)
    assert abs(L - L0) < 1e-12
    np.testing.assert_allclose(gC, gC0, rtol=1e-14)
    np.testing.assert_allclose(gD, gD0, rtol=1e-14)
    z = lo.masked_loss(rgb, depth, tgt, tdepth, np.zeros((26, 30), bool), 1.0, 0.2, 0.2)
    assert z[0] == 0.0 and not z[1].any() and not z[2].any()
