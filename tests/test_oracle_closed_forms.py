"""Pins of the FP64 oracle against closed forms, textbook routines and library functions.

Each test states what fixes the expected value independently of the oracle's code:
  * projection of an axis-aligned Gaussian (EWA Jacobian written by hand),
  * a single isotropic Gaussian's rendered peak, profile and footprint (lattice count),
  * the 0.99 alpha clamp and the 1/255 cutoff,
  * the transmittance product of stacked layers with early termination,
  * the SH basis against scipy's complex spherical harmonics and quadrature orthonormality,
  * the L1 loss and PSNR on constant images.
"""
import math

import numpy as np
import pytest

import synth


def one_gaussian(mu, log_scales, quat=(1, 0, 0, 0), logit=0.0, sh=None, degree=0):
    K = (degree + 1) ** 2
    shv = np.zeros((3 * K, 1)) if sh is None else np.asarray(sh, np.float64).reshape(3 * K, 1)
    return dict(means=np.asarray(mu, np.float64).reshape(3, 1), log_scales=np.asarray(log_scales, np.float64).reshape(3, 1),
                quats=np.asarray(quat, np.float64).reshape(4, 1), opacity_logits=np.array([logit], np.float64),
                sh=shv, sh_degree=degree)


def stack(gs):
    out = {k: np.concatenate([g[k] for g in gs], axis=-1) for k in ("means", "log_scales", "quats", "opacity_logits", "sh")}
    out["sh_degree"] = gs[0]["sh_degree"]
    return out


def cam(W, H, f=50.0, cx=None, cy=None, R=np.eye(3), t=np.zeros(3), bg=(0, 0, 0)):
    return synth.make_camera(R, t, f, f, W / 2.0 if cx is None else cx, H / 2.0 if cy is None else cy, W, H, bg=bg)


def logit(o):
    return math.log(o / (1 - o))


def test_projection_axis_aligned_on_axis(orc):
    # q = identity, mean on the optical axis: J = diag(f/z, f/z) in its first two columns, so
    # Sigma' = diag((fx e^sx / z)^2 + 0.3, (fy e^sy / z)^2 + 0.3) and (u, v) = (cx, cy).
    z, sx, sy, sz = 4.0, math.log(0.05), math.log(0.12), math.log(0.3)
    c = synth.make_camera(np.eye(3), np.zeros(3), 80.0, 90.0, 31.5, 20.5, 64, 40)
    p = orc.project(one_gaussian([0, 0, z], [sx, sy, sz]), c)
    assert p["visible"][0] == 1
    assert p["u"][0] == pytest.approx(31.5, abs=1e-12) and p["v"][0] == pytest.approx(20.5, abs=1e-12)
    exx = (80.0 * 0.05 / z) ** 2 + 0.3
    eyy = (90.0 * 0.12 / z) ** 2 + 0.3
    assert p["cov_xx"][0] == pytest.approx(exx, rel=1e-13)
    assert p["cov_yy"][0] == pytest.approx(eyy, rel=1e-13)
    assert abs(p["cov_xy"][0]) < 1e-15
    assert p["Qa"][0] == pytest.approx(1 / exx, rel=1e-13) and p["Qc"][0] == pytest.approx(1 / eyy, rel=1e-13)
    assert p["z"][0] == z


def test_projection_off_axis_jacobian(orc):
    # Isotropic sigma at (x, 0, z): J J^T = [[fx^2/z^2 + fx^2 x^2/z^4, 0], [0, fy^2/z^2]] (y = 0).
    x, z, s = 0.7, 3.0, 0.05
    fx, fy = 60.0, 70.0
    c = synth.make_camera(np.eye(3), np.zeros(3), fx, fy, 50.0, 40.0, 100, 80)
    p = orc.project(one_gaussian([x, 0, z], [math.log(s)] * 3), c)
    exx = s * s * (fx ** 2 / z ** 2 + fx ** 2 * x ** 2 / z ** 4) + 0.3
    eyy = s * s * fy ** 2 / z ** 2 + 0.3
    assert p["cov_xx"][0] == pytest.approx(exx, rel=1e-13)
    assert p["cov_yy"][0] == pytest.approx(eyy, rel=1e-13)
    assert p["u"][0] == pytest.approx(fx * x / z + 50.0, rel=1e-14)
    # beyond the guard band (|x/z| > 1.3 W / (2 fx)) the Jacobian uses the clamped ratio
    xg = 3.0 * z
    lim = 1.3 * 100 / (2 * fx)
    p2 = orc.project(one_gaussian([xg, 0, z], [math.log(s)] * 3), c)
    exx2 = s * s * (fx ** 2 / z ** 2 + fx ** 2 * lim ** 2 / z ** 2) + 0.3
    assert p2["cov_xx"][0] == pytest.approx(exx2, rel=1e-13)


def test_projection_rotated_anisotropic_matches_rotation_of_axes(orc):
    # A Gaussian rotated by 90 degrees about the optical axis swaps its x and y scales.
    sx, sy = math.log(0.2), math.log(0.05)
    c = cam(101, 101, f=100.0)
    q90 = (math.cos(math.pi / 4), 0, 0, math.sin(math.pi / 4))
    a = orc.project(one_gaussian([0, 0, 5], [sx, sy, -3]), c)
    b = orc.project(one_gaussian([0, 0, 5], [sx, sy, -3], quat=q90), c)
    assert b["cov_xx"][0] == pytest.approx(a["cov_yy"][0], rel=1e-12)
    assert b["cov_yy"][0] == pytest.approx(a["cov_xx"][0], rel=1e-12)
    # un-normalised quaternions give the same result (normalisation is part of the definition)
    b2 = orc.project(one_gaussian([0, 0, 5], [sx, sy, -3], quat=tuple(3.7 * v for v in q90)), c)
    assert b2["cov_xx"][0] == pytest.approx(b["cov_xx"][0], rel=1e-13)


def single_isotropic(orc, o, sigma_px, W=41, H=31, f=100.0, z=5.0, h_dc=(0.3, -0.2, 0.6)):
    # isotropic 3-D Gaussian on the optical axis; W, H odd so (cx, cy) = (W/2, H/2) is a pixel centre
    s = math.sqrt(max(sigma_px ** 2 - 0.3, 1e-12)) * z / f
    g = one_gaussian([0, 0, z], [math.log(s)] * 3, logit=logit(o), sh=h_dc)
    c = cam(W, H, f=f)
    return g, c, z


@pytest.mark.parametrize("o,sig", [(0.5, 2.0), (0.8, 1.3), (0.3, 4.5)])
def test_single_gaussian_profile_peak_and_footprint(orc, o, sig):
    g, c, z = single_isotropic(orc, o, sig)
    r = orc.render(g, c)
    W, H = c["width"], c["height"]
    rgb0 = 0.5 + np.array([0.3, -0.2, 0.6]) / (2 * math.sqrt(math.pi))  # SH degree 0 colour
    ii, jj = np.meshgrid(np.arange(W), np.arange(H))
    r2 = (ii + 0.5 - W / 2) ** 2 + (jj + 0.5 - H / 2) ** 2
    alpha = o * np.exp(-r2 / (2 * sig * sig))
    inside = alpha >= 1 / 255
    # exact lattice count of pixel centres in the alpha >= 1/255 disc
    assert (r["n"] > 0).sum() == inside.sum()
    assert inside.sum() == (r2 <= 2 * sig * sig * math.log(255 * o)).sum()
    a = np.where(inside, np.minimum(alpha, 0.99), 0.0)
    for ch in range(3):
        np.testing.assert_allclose(r["rgb"][ch], rgb0[ch] * a, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(r["depth"], z * a, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(r["alpha"], a, rtol=1e-12, atol=1e-15)
    # peak at the centre pixel = o * rgb
    cy, cx = H // 2, W // 2
    np.testing.assert_allclose(r["rgb"][:, cy, cx], o * rgb0, rtol=1e-13)


def test_alpha_clamp_at_099(orc):
    g, c, z = single_isotropic(orc, 0.999, 3.0)
    r = orc.render(g, c)
    rgb0 = 0.5 + np.array([0.3, -0.2, 0.6]) / (2 * math.sqrt(math.pi))
    cy, cx = c["height"] // 2, c["width"] // 2
    np.testing.assert_allclose(r["rgb"][:, cy, cx], 0.99 * rgb0, rtol=1e-14)
    assert r["alpha"][cy, cx] == pytest.approx(0.99, rel=1e-14)


def test_cutoff_single_pixel_and_empty(orc):
    # opacity just above 1/255 with a wide footprint: only the centre pixel passes the cutoff
    g, c, z = single_isotropic(orc, 1 / 255 * 1.0005, 1.0)
    r = orc.render(g, c)
    assert (r["n"] > 0).sum() == 1
    # below 1/255 nothing is drawn and no gradient flows
    g, c, z = single_isotropic(orc, 1 / 255 * 0.999, 5.0)
    r = orc.render(g, c)
    assert (r["n"] > 0).sum() == 0 and np.all(r["rgb"] == 0)
    G = np.ones((3, c["height"], c["width"]))
    b = orc.render_bwd(g, c, G, np.ones((c["height"], c["width"])))
    for k in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        assert np.all(b[k] == 0)
    assert np.all(b["pose"] == 0)


def test_transmittance_product_stacked_layers(orc):
    # n coincident identical layers with alpha = 0.95 at the centre pixel: 0.05^3 = 1.25e-4 >= 1e-4
    # but 0.05^4 < 1e-4, so exactly three composite.  C = rgb (1 - 0.05^3); D = 0.95 sum z_k 0.05^(k-1).
    zs = [3.0, 3.5, 4.25, 5.0, 6.0]
    gs = []
    for z in zs:
        s = 0.02 * z / 100.0
        gs.append(one_gaussian([0, 0, z], [math.log(s)] * 3, logit=logit(0.95), sh=(0.3, -0.2, 0.6)))
    g = stack(gs[::-1])  # index order opposite to depth order
    c = cam(21, 21, f=100.0)
    r = orc.render(g, c, pixels=[[10, 10]])
    rgb0 = 0.5 + np.array([0.3, -0.2, 0.6]) / (2 * math.sqrt(math.pi))
    assert r["n"][0] == 3
    np.testing.assert_allclose(r["rgb"][0], rgb0 * (1 - 0.05 ** 3), rtol=1e-13)
    np.testing.assert_allclose(r["depth"][0], 0.95 * sum(z * 0.05 ** k for k, z in enumerate(zs[:3])), rtol=1e-13)
    np.testing.assert_allclose(r["alpha"][0], 1 - 0.05 ** 3, rtol=1e-13)
    np.testing.assert_allclose(r["T"][0], 0.05 ** 3, rtol=1e-12)


def test_background_and_depth_have_no_background_term(orc):
    g, c, z = single_isotropic(orc, 0.6, 2.0)
    c["bg"] = np.array([0.2, 0.4, 0.6], np.float32)
    r = orc.render(g, c)
    # far from the Gaussian: pure background colour, zero depth (Eq. 8 has no background term)
    np.testing.assert_allclose(r["rgb"][:, 0, 0], [0.2, 0.4, 0.6], rtol=1e-7)
    assert r["depth"][0, 0] == 0.0
    cy, cx = c["height"] // 2, c["width"] // 2
    rgb0 = 0.5 + np.array([0.3, -0.2, 0.6]) / (2 * math.sqrt(math.pi))
    np.testing.assert_allclose(r["rgb"][:, cy, cx], 0.6 * rgb0 + 0.4 * np.asarray(c["bg"], np.float64), rtol=1e-13)


def _real_sh_scipy(l, m, dirs):
    from scipy.special import sph_harm_y
    th = np.arccos(np.clip(dirs[:, 2], -1, 1))
    ph = np.arctan2(dirs[:, 1], dirs[:, 0])
    # scipy's Y_l^m carries the Condon-Shortley phase; (-1)^m removes it
    if m == 0:
        return sph_harm_y(l, 0, th, ph).real
    y = sph_harm_y(l, abs(m), th, ph)
    if m > 0:
        return math.sqrt(2) * (-1) ** m * y.real
    return math.sqrt(2) * (-1) ** m * y.imag


def test_sh_basis_matches_scipy(orc):
    rng = np.random.default_rng(5)
    d = rng.standard_normal((50, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y, _ = orc.sh_basis(3, d)
    k = 0
    for l in range(4):
        for m in range(-l, l + 1):
            np.testing.assert_allclose(Y[:, k], _real_sh_scipy(l, m, d), rtol=1e-12, atol=1e-14)
            k += 1
    # degree 0: Y_00 = 1 / (2 sqrt(pi))
    assert Y[0, 0] == pytest.approx(1 / (2 * math.sqrt(math.pi)), rel=1e-15)


def test_sh_basis_orthonormal_by_quadrature(orc):
    # Gauss-Legendre in cos(theta) x uniform phi integrates polynomials of degree <= 19 exactly
    xg, wg = np.polynomial.legendre.leggauss(12)
    nphi = 24
    ph = np.arange(nphi) * 2 * np.pi / nphi
    ct, PH = np.meshgrid(xg, ph, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([(st * np.cos(PH)).ravel(), (st * np.sin(PH)).ravel(), ct.ravel()], 1)
    w = (wg[:, None] * np.full(nphi, 2 * np.pi / nphi)[None, :]).ravel()
    Y, dY = orc.sh_basis(3, d)
    G = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh_gradient_matches_finite_differences(orc):
    rng = np.random.default_rng(6)
    d = rng.standard_normal((5, 3))
    Y, dY = orc.sh_basis(3, d)  # polynomial gradient, valid off the sphere too
    h = 1e-6
    for r in range(3):
        e = np.zeros(3)
        e[r] = h
        Yp, _ = orc.sh_basis(3, d + e)
        Ym, _ = orc.sh_basis(3, d - e)
        np.testing.assert_allclose((Yp - Ym) / (2 * h), dY[:, :, r], rtol=1e-6, atol=1e-8)


def test_l1_loss_and_psnr_closed_forms(orc):
    H, W = 6, 7
    rgb = np.full((3, H, W), 0.75)
    tgt = np.full((3, H, W), 0.5)
    dep = np.full((H, W), 3.0)
    tdep = np.full((H, W), 2.0)
    loss, gC, gD = orc.l1_loss(rgb, dep, tgt, tdep, 0.2)
    assert loss == pytest.approx(3 * 0.25 + 0.2 * 1.0, rel=1e-15)
    np.testing.assert_allclose(gC, 1.0 / (H * W))
    np.testing.assert_allclose(gD, 0.2 / (H * W))
    # sign(0) = 0
    _, gC0, _ = orc.l1_loss(tgt, dep, tgt, None, 0.0)
    assert np.all(gC0 == 0)
    assert orc.psnr(rgb, tgt) == pytest.approx(10 * math.log10(1 / 0.0625), rel=1e-14)


def test_order_uses_float32_depth_key_then_index(orc):
    # Two coincident Gaussians whose depths differ by less than half a float32 ulp share the
    # depth key: the lower index composites first even though it is (in float64) farther away.
    z = 3.0
    a = one_gaussian([0, 0, z + 1e-8], [math.log(0.01)] * 3, logit=logit(0.6), sh=(1.0, 0.0, 0.0))
    b = one_gaussian([0, 0, z], [math.log(0.01)] * 3, logit=logit(0.3), sh=(0.0, 1.0, 0.0))
    c = cam(21, 21, f=100.0)
    r = orc.render(stack([a, b]), c, pixels=[[10, 10]])
    k = 1 / (2 * math.sqrt(math.pi))
    ca, cb = np.array([0.5 + k, 0.5, 0.5]), np.array([0.5, 0.5 + k, 0.5])
    np.testing.assert_allclose(r["rgb"][0], 0.6 * ca + 0.4 * 0.3 * cb, rtol=1e-13)
    # once the keys differ, depth decides
    a2 = one_gaussian([0, 0, z + 1e-5], [math.log(0.01)] * 3, logit=logit(0.6), sh=(1.0, 0.0, 0.0))
    r2 = orc.render(stack([a2, b]), c, pixels=[[10, 10]])
    np.testing.assert_allclose(r2["rgb"][0], 0.3 * cb + 0.7 * 0.6 * ca, rtol=1e-13)


def test_contributor_lists_by_brute_force(orc):
    # The composited list of a pixel, rebuilt by brute force from the (separately pinned)
    # projection: every Gaussian with o exp(-D^T Q D / 2) >= 1/255 at the pixel centre, ordered by
    # (float32 depth, index), composited front to back until T (1 - min(a, 0.99)) < 1e-4.
    g = synth.random_gaussians(11, 300, 0, xy_half=1.0, z_range=(2.0, 6.0), log_scale_mean=-2.0)
    c = cam(40, 30, f=40.0)
    pr = orc.project(g, c)
    rng = np.random.default_rng(5)
    pix = np.stack([rng.integers(0, 40, 60), rng.integers(0, 30, 60)], axis=1)
    lists = orc.contributors(g, c, pix)
    ren = orc.render(g, c, pixels=pix)
    checked = 0
    for k, (x, y) in enumerate(pix):
        vis = pr["visible"] > 0
        dx, dy = x + 0.5 - pr["u"], y + 0.5 - pr["v"]
        q = pr["Qa"] * dx * dx + 2 * pr["Qb"] * dx * dy + pr["Qc"] * dy * dy
        a = pr["opacity"] * np.exp(-0.5 * q)
        cand = np.nonzero(vis & (a >= 1 / 255))[0]
        if np.any(np.abs(a[vis] * 255 - 1) < 1e-9):
            continue  # knife edge
        cand = cand[np.lexsort((cand, pr["z"][cand].astype(np.float32)))]
        T, exp = 1.0, []
        for i in cand:
            ai = min(a[i], 0.99)
            if T * (1 - ai) < 1e-4:
                break
            exp.append(i)
            T *= 1 - ai
        assert list(lists[k]) == exp, (x, y)
        assert ren["n"][k] == len(exp)
        checked += 1
    assert checked > 50
    assert sum(len(x) for x in lists) > 100
