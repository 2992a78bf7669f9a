"""FP64 oracle of the supervision masks and the full training loss (Sec. III-C: Eq. 7 and
Eq. 9-12).  Test infrastructure only: the test-suite, the smoke check and the benchmark's CPU
baseline may use it; the product path never imports it.

Everything here is the plain definition, written with whole-image numpy operations and explicit
loops over window offsets (no separable filtering, no tiling):

* geometric support  M_geo(x) = [T_final(x) <= 1 - tau_geo], the comparison taken in float32
  (accumulated opacity 1 - T at least tau_geo);
* interior mask      M_int = Erode(M_geo, r) with the disk {dx^2 + dy^2 <= r^2}; pixels outside
  the image count as unsupported, so the erosion also trims an r-pixel frame (Eq. 7);
* Eq. 10 and 12      masked means of the channel-summed |C - C~| and of |D - D~| over M_int;
* Eq. 11             1 - SSIM of the images restricted to M_int: both images are set to zero
  outside the mask, the usual SSIM map (11x11 Gaussian window, sigma 1.5, zero padding
  at the image border, C1 = 0.01^2, C2 = 0.03^2 for unit dynamic range) is formed per channel,
  and SSIM is its mean over the pixels of M_int and the three channels;
* Eq. 9              lambda_rgb L_rgb + lambda_ssim L_ssim + lambda_depth L_depth per view; an
  empty mask gives a zero loss and zero gradient for that view.

The masks are piecewise constant in the render, so no gradient flows through them.
"""
from __future__ import annotations

import numpy as np

TAU_GEO = 0.5
R_ERODE = 2
SSIM_SIZE = 11
SSIM_SIGMA = 1.5
SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2


def disk_offsets(r):
    """Offsets (dy, dx) of the erosion disk of radius r."""
    return [(dy, dx) for dy in range(-r, r + 1) for dx in range(-r, r + 1) if dy * dy + dx * dx <= r * r]


def _shift(img, dy, dx, fill):
    """out[y, x] = img[y + dy, x + dx], or fill where that falls outside the image."""
    H, W = img.shape
    out = np.full_like(img, fill)
    ys, ye = max(0, -dy), min(H, H - dy)
    xs, xe = max(0, -dx), min(W, W - dx)
    if ys < ye and xs < xe:
        out[ys:ye, xs:xe] = img[ys + dy:ye + dy, xs + dx:xe + dx]
    return out


def support_masks(T_final, tau_geo=TAU_GEO, r_erode=R_ERODE):
    """Eq. 7 for one view: (M_geo, M_int) as bool [H, W] from the final transmittance [H, W]."""
    T = np.asarray(T_final, np.float32)
    thr = np.float32(1.0) - np.float32(tau_geo)
    geo = T <= thr
    inner = np.ones_like(geo)
    for dy, dx in disk_offsets(r_erode):
        inner &= _shift(geo, dy, dx, False)
    return geo, inner


def gaussian_window(size=SSIM_SIZE, sigma=SSIM_SIGMA):
    """The normalised 2-D Gaussian window w[dy + r, dx + r] (outer product of the 1-D taps)."""
    k = np.arange(size, dtype=np.float64) - size // 2
    g = np.exp(-k * k / (2.0 * sigma * sigma))
    g /= g.sum()
    return np.outer(g, g)


def window_mean(img, w):
    """out[y, x] = sum_d w[d] img[(y, x) + d] with img = 0 outside the image."""
    r = w.shape[0] // 2
    out = np.zeros(img.shape, np.float64)
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            out += w[dy + r, dx + r] * _shift(img, dy, dx, 0.0)
    return out


def window_mean_adjoint(g, w):
    """Adjoint of window_mean: in_bar[q] = sum_d w[d] g[q - d] (g = 0 outside the image)."""
    r = w.shape[0] // 2
    out = np.zeros(g.shape, np.float64)
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            out += w[dy + r, dx + r] * _shift(g, -dy, -dx, 0.0)
    return out


def ssim_terms(X, Y, w=None):
    """Window statistics and the SSIM map of one channel (float64 [H, W] each)."""
    w = gaussian_window() if w is None else w
    mx, my = window_mean(X, w), window_mean(Y, w)
    exx, eyy, exy = window_mean(X * X, w), window_mean(Y * Y, w), window_mean(X * Y, w)
    vx, vy, cxy = exx - mx * mx, eyy - my * my, exy - mx * my
    n1, d1 = 2 * mx * my + SSIM_C1, mx * mx + my * my + SSIM_C1
    n2, d2 = 2 * cxy + SSIM_C2, vx + vy + SSIM_C2
    lum, cs = n1 / d1, n2 / d2
    return dict(mx=mx, my=my, vx=vx, vy=vy, cxy=cxy, d1=d1, d2=d2, lum=lum, cs=cs, S=lum * cs)


def ssim_loss(rgb, target, mask, want_grad=True):
    """Eq. 11 for one view: L = 1 - (1/(3|M|)) sum_{x in M} sum_c S_c(x) on the mask-restricted
    images.  rgb, target [3, H, W]; mask bool [H, W].  Returns (L, dL/drgb [3, H, W])."""
    rgb, target = np.asarray(rgb, np.float64), np.asarray(target, np.float64)
    M = np.asarray(mask, bool)
    cnt = int(M.sum())
    grad = np.zeros(rgb.shape)
    if cnt == 0:
        return 0.0, grad
    Mf = M.astype(np.float64)
    w = gaussian_window()
    total = 0.0
    for c in range(3):
        X, Y = np.where(M, rgb[c], 0.0), np.where(M, target[c], 0.0)
        t = ssim_terms(X, Y, w)
        total += t["S"][M].sum()
        if not want_grad:
            continue
        # dS/d(window mean of x), dS/d(window mean of x^2), dS/d(window mean of x y): the
        # variance and covariance are E[x^2] - mx^2 and E[xy] - mx my.
        dlum_dmx = 2.0 * (t["my"] - t["mx"] * t["lum"]) / t["d1"]
        dcs_dmx = 2.0 * (t["mx"] * t["cs"] - t["my"]) / t["d2"]
        a = t["cs"] * dlum_dmx + t["lum"] * dcs_dmx
        b = -t["S"] / t["d2"]
        e = 2.0 * t["lum"] / t["d2"]
        scale = -Mf / (3.0 * cnt)  # dL/dS_c(x)
        gX = (window_mean_adjoint(scale * a, w) + 2.0 * X * window_mean_adjoint(scale * b, w)
              + Y * window_mean_adjoint(scale * e, w))
        grad[c] = np.where(M, gX, 0.0)
    return 1.0 - total / (3.0 * cnt), grad


def masked_loss(rgb, depth, target_rgb, target_depth, mask, lambda_rgb=1.0, lambda_ssim=0.0,
                lambda_depth=0.0):
    """Eq. 9 with Eq. 10-12 for one view.  mask bool [H, W] (None = all ones); target_depth may
    be None (no depth term).  Returns (L, dL/drgb [3, H, W], dL/ddepth [H, W]); sign(0) = 0."""
    rgb, t = np.asarray(rgb, np.float64), np.asarray(target_rgb, np.float64)
    H, W = rgb.shape[1:]
    M = np.ones((H, W), bool) if mask is None else np.asarray(mask, bool)
    cnt = int(M.sum())
    gC = np.zeros(rgb.shape)
    gD = np.zeros((H, W))
    if cnt == 0:
        return 0.0, gC, gD
    dC = rgb - t
    loss = lambda_rgb * np.abs(dC[:, M]).sum() / cnt
    gC += np.where(M, lambda_rgb * np.sign(dC) / cnt, 0.0)
    if target_depth is not None and lambda_depth != 0.0:
        dD = np.asarray(depth, np.float64) - np.asarray(target_depth, np.float64)
        loss += lambda_depth * np.abs(dD[M]).sum() / cnt
        gD = np.where(M, lambda_depth * np.sign(dD) / cnt, 0.0)
    if lambda_ssim != 0.0:
        ls, gs = ssim_loss(rgb, t, M)
        loss += lambda_ssim * ls
        gC += lambda_ssim * gs
    return loss, gC, gD
