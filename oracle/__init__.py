"""FP64 CPU oracle of the Gaussian-splatting rasterizer (test infrastructure only).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may import this
package.  The product path (``paper_2604_12942_amd``) never imports it and shares no code with
it; the two meet only through the seeded inputs drawn by ``synth``.

The compiled part lives in ``gsr_oracle.c`` (plain C, double precision, OpenMP over pixels).
This module marshals numpy arrays into it and adds the loss, PSNR and Adam definitions of the
paper's Sec. III-C (Eq. 9, 10 and 12 with the all-ones mask; the sparse optimizer).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gsr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_gsr.so")
_lib = None


def build(force=True):
    """Compile the oracle with gcc (no GPU involved)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Cam(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("t", C.c_double * 3), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("z_near", C.c_double), ("bg", C.c_double * 3),
                ("width", C.c_int32), ("height", C.c_int32)]


class _Gauss(C.Structure):
    _fields_ = [("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity_logits", C.c_void_p), ("sh", C.c_void_p), ("n", C.c_int64),
                ("sh_degree", C.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        P = C.c_void_p
        L.orc_sh_basis.argtypes = [C.c_int, P, P, P]
        L.orc_sh_basis.restype = C.c_int
        L.orc_project.argtypes = [C.POINTER(_Gauss), C.POINTER(_Cam), P]
        L.orc_render.argtypes = [C.POINTER(_Gauss), C.POINTER(_Cam), P, C.c_int64, P, P, P, P, P]
        L.orc_render_bwd.argtypes = [C.POINTER(_Gauss), C.POINTER(_Cam), P, P, P, P, P, P, P, P, P,
                                     C.c_double, P, P]
        L.orc_render_bwd.restype = C.c_int64
        L.orc_num_threads.restype = C.c_int
        L.orc_contributors.argtypes = [C.POINTER(_Gauss), C.POINTER(_Cam), P, C.c_int64, C.c_int64, P, P]
        L.orc_adam.argtypes = [P, P, P, P, C.c_int64, C.c_int64, P, C.c_double, C.c_double, C.c_double,
                               C.c_double, C.c_int]
        _lib = L
    return _lib


def num_threads():
    """Threads the oracle's OpenMP loops run on."""
    return int(lib().orc_num_threads())


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, np.float64)


class _Bound:
    """Keeps the float64 copies alive for the duration of a call."""

    def __init__(self, g):
        self.arrs = [_f64(g["means"]), _f64(g["log_scales"]), _f64(g["quats"]),
                     _f64(g["opacity_logits"]), _f64(g["sh"])]
        n = self.arrs[0].shape[1]
        self.s = _Gauss(*[a.ctypes.data for a in self.arrs], n, int(g["sh_degree"]))
        self.n = n


def _cam(c):
    s = _Cam()
    s.R[:] = [float(v) for v in np.asarray(c["R"], np.float64).ravel()]
    s.t[:] = [float(v) for v in np.asarray(c["t"], np.float64).ravel()]
    s.fx, s.fy, s.cx, s.cy = float(c["fx"]), float(c["fy"]), float(c["cx"]), float(c["cy"])
    s.z_near = float(c.get("z_near", 0.2))
    s.bg[:] = [float(v) for v in np.asarray(c.get("bg", (0, 0, 0)), np.float64).ravel()]
    s.width, s.height = int(c["width"]), int(c["height"])
    return s


def sh_basis(degree, dirs):
    """Real SH basis Y[k] (and polynomial gradients) at unit directions dirs (m, 3)."""
    dirs = _f64(dirs).reshape(-1, 3)
    K = (degree + 1) ** 2
    Y = np.zeros((dirs.shape[0], K))
    dY = np.zeros((dirs.shape[0], 16, 3))
    for k in range(dirs.shape[0]):
        y = np.zeros(16)
        d = np.zeros((16, 3))
        lib().orc_sh_basis(degree, _ptr(np.ascontiguousarray(dirs[k])), _ptr(y), _ptr(d))
        Y[k] = y[:K]
        dY[k] = d
    return Y, dY[:, :K]


PROJ_FIELDS = ("visible", "u", "v", "z", "Qa", "Qb", "Qc", "opacity", "r", "g", "b",
               "cov_xx", "cov_xy", "cov_yy", "guard_margin", "sh_margin")


def project(g, cam):
    b = _Bound(g)
    out = np.zeros((b.n, 16))
    lib().orc_project(C.byref(b.s), C.byref(_cam(cam)), _ptr(out))
    return {k: out[:, j] for j, k in enumerate(PROJ_FIELDS)}


def render(g, cam, pixels=None):
    """Render every pixel (pixels=None) or the listed (x, y) pixel centres.

    Returns dict rgb ([3,H,W] or [m,3]), depth, T (final transmittance), n (contributors),
    margin (smallest relative decision margin; below ~1e-5 the pixel is a knife edge)."""
    b = _Bound(g)
    W, H = int(cam["width"]), int(cam["height"])
    if pixels is None:
        m = W * H
        rgb = np.zeros((3, H, W))
        shp = (H, W)
        pix = None
    else:
        pix = np.ascontiguousarray(pixels, np.int32).reshape(-1, 2)
        m = pix.shape[0]
        rgb = np.zeros((m, 3))
        shp = (m,)
    depth = np.zeros(shp)
    T = np.zeros(shp)
    n = np.zeros(shp, np.int32)
    mg = np.zeros(shp)
    lib().orc_render(C.byref(b.s), C.byref(_cam(cam)), _ptr(pix), m, _ptr(rgb), _ptr(depth), _ptr(T),
                     _ptr(n), _ptr(mg))
    return dict(rgb=rgb, depth=depth, T=T, alpha=1.0 - T, n=n, margin=mg)


def contributors(g, cam, pixels, cap=4096):
    """Composited Gaussian indices of each (x, y) in pixels, front to back: a list of int64 arrays."""
    b = _Bound(g)
    pix = np.ascontiguousarray(np.asarray(pixels, np.int32).reshape(-1, 2))
    ids = np.zeros((pix.shape[0], cap), np.int64)
    counts = np.zeros(pix.shape[0], np.int32)
    lib().orc_contributors(C.byref(b.s), C.byref(_cam(cam)), _ptr(pix), pix.shape[0], cap, _ptr(ids), _ptr(counts))
    if np.any(counts > cap):
        raise ValueError("more than cap contributors at a pixel")
    return [ids[k, :counts[k]].copy() for k in range(pix.shape[0])]


def render_bwd(g, cam, dL_drgb, dL_ddepth=None, knife_tol=1e-5, want_pose=True):
    """Gradient of L = <dL_drgb, C> + <dL_ddepth, D> w.r.t. every parameter and the camera pose
    (left se(3) perturbation, (rho, phi)).  Returns dict of float64 arrays in input layouts plus
    'pose' (6,), 'screen' [n,10] (u, v, Qa, Qb, Qc, o, r, g, b, z), 'knife_px' [H,W] bool,
    'knife_g' [n] bool and 'n_knife'."""
    b = _Bound(g)
    n = b.n
    W, H = int(cam["width"]), int(cam["height"])
    out = dict(means=np.zeros((3, n)), log_scales=np.zeros((3, n)), quats=np.zeros((4, n)),
               opacity_logits=np.zeros(n), sh=np.zeros_like(b.arrs[4]))
    pose = np.zeros(6)
    screen = np.zeros((n, 10))
    kp = np.zeros((H, W), np.uint8)
    kg = np.zeros(n, np.uint8)
    gr = _f64(dL_drgb)
    gd = _f64(dL_ddepth) if dL_ddepth is not None else None
    nk = lib().orc_render_bwd(C.byref(b.s), C.byref(_cam(cam)), _ptr(gr), _ptr(gd), _ptr(out["means"]),
                              _ptr(out["log_scales"]), _ptr(out["quats"]), _ptr(out["opacity_logits"]),
                              _ptr(out["sh"]), _ptr(pose) if want_pose else None, _ptr(screen),
                              float(knife_tol), _ptr(kp), _ptr(kg))
    out.update(pose=pose, screen=screen, knife_px=kp.astype(bool), knife_g=kg.astype(bool), n_knife=int(nk))
    return out


def l1_loss(rgb, depth, target_rgb, target_depth, lambda_depth):
    """Eq. 9/10/12 with the all-ones mask: mean over pixels of the channel-summed |C - C~| plus
    lambda_depth times the mean of |D - D~|.  Returns (loss, dL/dC, dL/dD); sign(0) = 0."""
    rgb, t = _f64(rgb), _f64(target_rgb)
    P = rgb.shape[-1] * rgb.shape[-2]
    dC = rgb - t
    loss = np.abs(dC).sum() / P
    gC = np.sign(dC) / P
    gD = np.zeros(rgb.shape[-2:])
    if target_depth is not None and lambda_depth != 0.0:
        dD = _f64(depth) - _f64(target_depth)
        loss += lambda_depth * np.abs(dD).sum() / P
        gD = lambda_depth * np.sign(dD) / P
    return loss, gC, gD


def psnr(rgb, target):
    """PSNR = 10 log10(1 / MSE) with the render clamped to [0, 1] for the metric."""
    mse = np.mean((np.clip(_f64(rgb), 0, 1) - _f64(target)) ** 2)
    return 10.0 * np.log10(1.0 / mse)


def adam(param, grad, m, v, mask, lr, beta1=0.9, beta2=0.999, eps=1e-15, step=1):
    """Sparse Adam on [cols, rows] arrays in place (float64); rows with mask 0 keep p, m, v."""
    arrs = [np.ascontiguousarray(a, np.float64) for a in (param, grad, m, v)]
    if arrs[0].ndim == 1:
        arrs = [a.reshape(1, -1) for a in arrs]
    cols, rows = arrs[0].shape
    mk = np.ascontiguousarray(mask, np.uint8) if mask is not None else None
    lib().orc_adam(*[_ptr(a) for a in arrs], rows, cols, _ptr(mk), lr, beta1, beta2, eps, step)
    return arrs
