"""FP64 oracle of the point network that predicts Gaussian attributes per voxel for the model
branch of the cascaded initialisation (Sec. III-B, Eq. 3: the feed-forward prediction Theta_model;
here a per-voxel point network stands in for the paper's image model).

TEST INFRASTRUCTURE ONLY (imported by tests and the benchmark's CPU leg, never by the product
path).  Plain numpy in double precision with BF16 rounding applied at the same points as on the
GPU: weights and every GEMM input, round to nearest even from float32.  Bias, ReLU and accumulation
are not rounded.

Network (readings; the paper's own model is an image network that is not reproduced):
  per point  x = (p - mu) / 0.5 m  (a voxel's fitting points repeated cyclically to 32 rows)
  3 -> 64 -> 64 -> 64 with ReLU, shared over points; max over the 32 rows (ties: lowest row)
  concat 12 voxel features: log(max(lambda, (5 mm)^2) / 0.5^2) ascending, then v_min, v_mid, v_max
  76 -> 64 with ReLU, 64 -> 8 = (log-scales s[3], quaternion q[4], opacity logit omega)
Training loss per voxel (mean over voxels):
  KL(N(0, Sigma_pred) || N(0, Sigma_tgt)) + 0.1 |sigmoid(omega) - o_tgt|,
  Sigma_pred = R(q / |q|) diag(exp(2 s)) R(q / |q|)^T.
Backward GEMMs round their inputs (upstream gradients too) to BF16 when round_grads is set.
"""
from __future__ import annotations

import numpy as np

ROWS = 32
WIDTH = 64
N_FEAT = 12
N_OUT = 8
LAYERS = (("W1", "b1", 3, WIDTH), ("W2", "b2", WIDTH, WIDTH), ("W3", "b3", WIDTH, WIDTH),
          ("W4", "b4", WIDTH + N_FEAT, WIDTH), ("W5", "b5", WIDTH, N_OUT))
LAMBDA_FLOOR = 0.005 ** 2


def bf16(x):
    """Round to bfloat16 (kept in float64): to float32 by round-to-nearest-even, then the upper
    16 bits of the float32 pattern by round-to-nearest-even."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    out = u.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(nan, np.nan, out)


def init_weights(seed):
    """He-uniform weights, zero biases (float32 master copies)."""
    rng = np.random.default_rng(seed)
    W = {}
    for w, b, k, n in LAYERS:
        lim = np.sqrt(6.0 / k)
        W[w] = rng.uniform(-lim, lim, (k, n)).astype(np.float32)
        W[b] = np.zeros(n, np.float32)
    return W


def voxel_inputs(points, vox):
    """Per voxel: the 32 input rows (fitting points repeated cyclically, centred and scaled) and
    the 12 features.  points [N, 3]; vox from init_oracle.voxel_pca."""
    P = np.asarray(points, np.float64)
    nv = len(vox["n"])
    X = np.zeros((nv, ROWS, 3))
    for v in range(nv):
        ids = np.asarray(vox["ids"][v])
        rows = ids[np.arange(ROWS) % len(ids)]
        X[v] = (P[rows] - vox["mu"][v]) / 0.5
    lam = np.maximum(vox["evals"], LAMBDA_FLOOR)
    R = vox["R"]  # columns v_max, v_mid, v_min
    F = np.concatenate([np.log(lam / 0.25), R[:, :, 2], R[:, :, 1], R[:, :, 0]], axis=1)
    return X, F


U32 = 2.0 ** -24  # float32 unit roundoff


class Jitter:
    """Knife-edge screen for the BF16 rounding points (test infrastructure, off by default).

    A float32 evaluation of a sum of K terms in another order differs from the exact sum by at
    most about K u S (u = 2^-24, S = the sum of the terms' magnitudes).  Where the exact value lies
    that close to a BF16 rounding midpoint, the rounded value, and everything computed from it,
    can differ by one BF16 step.  One Jitter realisation moves every value at a rounding point by
    an independent uniform amount in [-c K u S, c K u S] before rounding (and before the ReLU
    decision that precedes it); elements that move by more than a fraction of the parity
    tolerance across a few seeded realisations are knife edges."""

    def __init__(self, seed, c=1.0):
        self.rng = np.random.default_rng(seed)
        self.c = c

    def __call__(self, a, K, S):
        return a + self.rng.uniform(-1.0, 1.0, a.shape) * (self.c * K * U32) * S


def _dense(x, w, b, jit):
    """x @ w + b, moved by one jitter realisation if given."""
    a = x @ w + b
    if jit is not None:
        a = jit(a, w.shape[0] + 1, np.abs(x) @ np.abs(w) + np.abs(b))
    return a


def forward(W, X, F, keep=False, jitter=None):
    """Outputs [nv, 8]; with keep, also the intermediates the backward needs.  jitter: a Jitter
    (knife-edge screen only; None for the definition)."""
    Wb = {k: bf16(W[k]) for k, _, _, _ in LAYERS}
    b = {bk: np.asarray(W[bk], np.float64) for _, bk, _, _ in LAYERS}
    X = np.asarray(X, np.float64)
    F = np.asarray(F, np.float64)
    if jitter is not None:
        X = jitter(X, 1, np.abs(X))
        F = jitter(F, 2, np.abs(F))
    x = bf16(X)                                   # [nv, 32, 3]
    a1 = _dense(x, Wb["W1"], b["b1"], jitter)
    h1 = bf16(np.maximum(a1, 0))
    a2 = _dense(h1, Wb["W2"], b["b2"], jitter)
    h2 = bf16(np.maximum(a2, 0))
    a3 = _dense(h2, Wb["W3"], b["b3"], jitter)
    h3 = np.maximum(a3, 0)
    arg = np.argmax(h3, axis=1)                   # first maximum = lowest row on ties
    g = np.take_along_axis(h3, arg[:, None, :], axis=1)[:, 0, :]
    z = bf16(np.concatenate([g, F], axis=1))      # [nv, 76]
    a4 = _dense(z, Wb["W4"], b["b4"], jitter)
    h4 = bf16(np.maximum(a4, 0))
    y = h4 @ Wb["W5"] + b["b5"]
    if not keep:
        return y
    return y, dict(x=x, a1=a1, h1=h1, a2=a2, h2=h2, a3=a3, arg=arg, z=z, a4=a4, h4=h4, Wb=Wb)


def quat_to_rot(q):
    """Unit quaternions (w, x, y, z) [n, 4] -> rotation matrices [n, 3, 3]."""
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    return np.stack([np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
                     np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
                     np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], 1)


def drot_dquat(q):
    """d R_ab / d q_c for unit-quaternion entries (treating q as free) [n, 3, 3, 4]."""
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    n = q.shape[0]
    D = np.zeros((n, 3, 3, 4))
    # row 0
    D[:, 0, 0] = np.stack([0 * w, 0 * w, -4 * y, -4 * z], -1)
    D[:, 0, 1] = np.stack([-2 * z, 2 * y, 2 * x, -2 * w], -1)
    D[:, 0, 2] = np.stack([2 * y, 2 * z, 2 * w, 2 * x], -1)
    # row 1
    D[:, 1, 0] = np.stack([2 * z, 2 * y, 2 * x, 2 * w], -1)
    D[:, 1, 1] = np.stack([0 * w, -4 * x, 0 * w, -4 * z], -1)
    D[:, 1, 2] = np.stack([-2 * x, -2 * w, 2 * z, 2 * y], -1)
    # row 2
    D[:, 2, 0] = np.stack([-2 * y, 2 * z, -2 * w, 2 * x], -1)
    D[:, 2, 1] = np.stack([2 * x, 2 * w, 2 * z, 2 * y], -1)
    D[:, 2, 2] = np.stack([0 * w, -4 * x, -4 * y, 0 * w], -1)
    return D


def loss(y, cov_t, o_t):
    """Mean over voxels of KL(N(0, Sigma_pred) || N(0, Sigma_tgt)) + 0.1 |sigmoid(omega) - o_t|,
    and its gradient with respect to y.  cov_t [nv, 3, 3] SPD, o_t [nv]."""
    nv = y.shape[0]
    s, q, om = y[:, :3], y[:, 3:7], y[:, 7]
    qn = np.linalg.norm(q, axis=1, keepdims=True)
    qh = q / qn
    R = quat_to_rot(qh)
    A = np.linalg.inv(cov_t)
    e2s = np.exp(2 * s)
    Sp = R @ (e2s[:, :, None] * np.transpose(R, (0, 2, 1)))
    kl = 0.5 * (np.einsum("nij,nji->n", A, Sp) - 3 + np.log(np.linalg.det(cov_t)) - 2 * s.sum(1))
    sg = 1 / (1 + np.exp(-om))
    L = np.mean(kl + 0.1 * np.abs(sg - o_t))
    # gradients (per voxel, then / nv)
    AR = A @ R                                   # columns A r_j
    rAr = np.einsum("nij,nij->nj", R, AR)        # r_j^T A r_j
    ds = e2s * rAr - 1.0
    dR = AR * e2s[:, None, :]                    # dKL/dR[:, j] = e^{2 s_j} A r_j
    dqh = np.einsum("nab,nabc->nc", dR, drot_dquat(qh))
    dq = (dqh - qh * np.sum(qh * dqh, axis=1, keepdims=True)) / qn
    dom = 0.1 * np.sign(sg - o_t) * sg * (1 - sg)
    dy = np.concatenate([ds, dq, dom[:, None]], axis=1) / nv
    return L, dy


def backward(W, keep, dy, round_grads=True, jitter=None):
    """Gradients of the parameters given dL/dy [nv, 8] and forward(..., keep=True)'s record.
    jitter: a Jitter applied to every value before its BF16 rounding (knife-edge screen only)."""
    r = bf16 if round_grads else (lambda a: a)

    def dmat(g, w):  # g @ w.T, jittered like a forward layer
        d = g @ w.T
        if jitter is not None:
            d = jitter(d, w.shape[1], np.abs(g) @ np.abs(w.T))
        return d

    Wb = keep["Wb"]
    G = {}
    dyr = r(dy if jitter is None else jitter(dy, 4, np.abs(dy)))
    G["W5"] = np.einsum("nk,nj->kj", keep["h4"], dyr)
    G["b5"] = dy.sum(0)
    dh4 = dmat(dyr, Wb["W5"])
    da4 = dh4 * (keep["a4"] > 0)
    da4r = r(da4)
    G["W4"] = np.einsum("nk,nj->kj", keep["z"], da4r)
    G["b4"] = da4.sum(0)
    dz = dmat(da4r, Wb["W4"])
    dg = dz[:, :WIDTH]
    nv = dy.shape[0]
    dh3 = np.zeros((nv, ROWS, WIDTH))
    np.put_along_axis(dh3, keep["arg"][:, None, :], dg[:, None, :], axis=1)
    da3 = dh3 * (keep["a3"] > 0)
    da3r = r(da3)
    G["W3"] = np.einsum("nrk,nrj->kj", keep["h2"], da3r)
    G["b3"] = da3.sum((0, 1))
    dh2 = dmat(da3r, Wb["W3"])
    da2 = dh2 * (keep["a2"] > 0)
    da2r = r(da2)
    G["W2"] = np.einsum("nrk,nrj->kj", keep["h1"], da2r)
    G["b2"] = da2.sum((0, 1))
    dh1 = dmat(da2r, Wb["W2"])
    da1 = dh1 * (keep["a1"] > 0)
    G["W1"] = np.einsum("nrk,nrj->kj", keep["x"], r(da1))
    G["b1"] = da1.sum((0, 1))
    return G


def knife_spread(W, X, F, realisations=12, seed=0, cov_t=None, o_t=None):
    """Largest change of every output (and, with targets, of every weight gradient of the
    training loss) over seeded Jitter realisations of the forward (and backward): the yardstick
    of the BF16 knife-edge screen.  Returns (y_spread [nv, 8], grad_spread dict or None)."""
    y0, k0 = forward(W, X, F, keep=True)
    G0 = None
    if cov_t is not None:
        _, dy0 = loss(y0, cov_t, o_t)
        G0 = backward(W, k0, dy0)
    ys = np.zeros_like(y0)
    gs = {k: np.zeros_like(v) for k, v in G0.items()} if G0 is not None else None
    for j in range(realisations):
        jit = Jitter(seed * 1000 + j)
        y, kp = forward(W, X, F, keep=True, jitter=jit)
        ys = np.maximum(ys, np.abs(y - y0))
        if G0 is not None:
            _, dy = loss(y, cov_t, o_t)
            G = backward(W, kp, dy, jitter=jit)
            for k in gs:
                gs[k] = np.maximum(gs[k], np.abs(G[k] - G0[k]))
    return ys, gs


def targets_from_gaussians(vox, gauss_log_scales, gauss_quats, gauss_logits, point_ids):
    """Per-voxel training targets: the mean covariance and mean opacity of the optimised Gaussians
    seeded from the voxel's points (point_ids[i] = the point Gaussian i was seeded from)."""
    nv = len(vox["n"])
    q = gauss_quats.T / np.linalg.norm(gauss_quats.T, axis=1, keepdims=True)
    R = quat_to_rot(q)
    S = np.exp(2 * gauss_log_scales.T)
    cov = R @ (S[:, :, None] * np.transpose(R, (0, 2, 1)))
    op = 1 / (1 + np.exp(-gauss_logits))
    v = vox["voxel"][point_ids]
    cnt = np.bincount(v, minlength=nv).astype(np.float64)
    ct = np.zeros((nv, 3, 3))
    np.add.at(ct, v, cov)
    ot = np.bincount(v, weights=op, minlength=nv)
    has = cnt > 0
    ct[has] /= cnt[has, None, None]
    ot[has] /= cnt[has]
    return ct, ot, has
