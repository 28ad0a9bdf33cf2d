"""CPU emulation of the low-precision MLP evaluators, written from their definitions.

Used to check that each GPU precision path computes the model it claims to (packing,
operand layouts, scales), not as a parity reference for the Monte Carlo itself, which is
the FP64 oracle's job.

Definitions (all precisions): with y = -log2(e) z, silu(z) = -ln(2) y / (1 + 2^y); the
kernels evaluate
    y1 = A0 x + c0,   h1 = y1 / (1 + 2^y1),
    y2 = A1 q(h1) + c1,   h2 = y2 / (1 + 2^y2),   E = b2 + w2' . h2
with A0 = q(-log2(e) W0), A1 = q(W1), c = -log2(e) b, w2' = -ln(2) W2, and q() the
precision's quantiser:
    fp32   : identity;
    bf16   : round to BF16 (nearest even);
    bf16x3 : hi = bf16(v), lo = bf16(v - hi); products hi*hi + hi*lo + lo*hi;
    fp8    : OCP E4M3 with power-of-two per-layer scales 2^k, k = ceil(log2(amax / 448));
             the activation scale bounds |h1| from the weights.
"""
from __future__ import annotations

import math

import numpy as np
import torch

L2E = np.float32(1.4426950408889634)
LN2 = np.float32(0.6931471805599453)


def split_params(p, n_in=108, H=128):
    p = np.asarray(p, dtype=np.float32)
    o = 0
    W0 = p[o:o + H * n_in].reshape(H, n_in); o += H * n_in
    b0 = p[o:o + H]; o += H
    W1 = p[o:o + H * H].reshape(H, H); o += H * H
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H]; o += H
    b2 = p[o]
    return W0, b0, W1, b1, W2, b2


def bf16(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16).float().numpy()


def e4m3(a):
    t = torch.from_numpy(np.clip(np.asarray(a, dtype=np.float32), -448.0, 448.0))
    return t.to(torch.float8_e4m3fn).float().numpy()


def _pow2_at_least(x):
    return 0 if x <= 0 else int(math.ceil(math.log2(x)))


def fp8_scales(params):
    W0, b0, W1, b1, W2, b2 = split_params(params)
    W0s = (-L2E * W0).astype(np.float32)
    k0 = _pow2_at_least(float(np.abs(W0s).max()) / 448.0)
    k1 = _pow2_at_least(float(np.abs(W1).max()) / 448.0)
    zmax = b0.astype(np.float64) + np.sum(
        np.maximum(0.0, W0.astype(np.float64).reshape(128, 27, 4).max(axis=2)), axis=1)
    hmax = float(np.max(1.4426950408889634 * np.maximum(zmax, 0.2785)))
    kh = _pow2_at_least(hmax / 448.0)
    return k0, k1, kh


def act(y):
    y = y.astype(np.float32)
    return (y / (np.float32(1.0) + np.exp2(y))).astype(np.float32)


def energies(params, X, prec):
    """Local energies of rows X [n, 108] (0/1 features) in the named precision."""
    W0, b0, W1, b1, W2, b2 = split_params(params)
    X = np.asarray(X, dtype=np.float64)
    W0s = (-L2E * W0).astype(np.float32)
    c0 = (-L2E * b0).astype(np.float32)
    c1 = (-L2E * b1).astype(np.float32)
    w2s = (-LN2 * W2).astype(np.float32)
    f64 = np.float64
    # FP32/BF16 paths carry the layer-0 bias as a weight column (quantised like the weights);
    # FP8 keeps it in FP32 as the accumulator's initial value
    if prec == "fp32":
        y1 = X @ W0s.T.astype(f64) + c0
        h = act(y1.astype(np.float32))
        y2 = h.astype(f64) @ W1.T.astype(f64) + c1
    elif prec == "bf16":
        y1 = X @ bf16(W0s).T.astype(f64) + bf16(c0)
        h = bf16(act(y1.astype(np.float32)))
        y2 = h.astype(f64) @ bf16(W1).T.astype(f64) + c1
    elif prec == "bf16x3":
        hi0 = bf16(W0s)
        lo0 = bf16(W0s - hi0)
        c0h = bf16(c0)
        c0 = c0h.astype(f64) + bf16(c0 - c0h)
        y1 = X @ (hi0.astype(f64) + lo0).T + c0
        h = act(y1.astype(np.float32))
        hh = bf16(h)
        hl = bf16(h - hh)
        A1h = bf16(W1)
        A1l = bf16(W1 - A1h)
        y2 = hh.astype(f64) @ A1h.T + hl.astype(f64) @ A1h.T + hh.astype(f64) @ A1l.T + c1
    elif prec == "fp8":
        k0, k1, kh = fp8_scales(params)
        A0 = e4m3(W0s * 2.0 ** -k0) * 2.0 ** k0
        A1 = e4m3(W1 * 2.0 ** -k1) * 2.0 ** k1
        y1 = X @ A0.T.astype(f64) + c0
        h = e4m3(act(y1.astype(np.float32)) * np.float32(2.0 ** -kh)) * 2.0 ** kh
        y2 = h.astype(f64) @ A1.T.astype(f64) + c1
    else:
        raise ValueError(prec)
    h2 = act(y2.astype(np.float32))
    return b2 + h2.astype(f64) @ w2s.astype(f64)


def dsilu_from_y(y):
    """silu'(z) with z = -ln(2) y: sigma (1 + z (1 - sigma)), sigma = 1 / (1 + 2^y)."""
    y = np.asarray(y, dtype=np.float32)
    sg = (np.float32(1.0) / (np.float32(1.0) + np.exp2(y))).astype(np.float32)
    z = (-LN2 * y).astype(np.float32)
    return (sg * (np.float32(1.0) + z * (np.float32(1.0) - sg))).astype(np.float32)


def fit_grad_bf16(params, X, g_rows):
    """Gradient sum_r g_r dE_r/dparams as the BF16 matrix-core backward defines it: each row's
    gradient is formed with a unit upstream gradient and then weighted by g_r (the kernel
    forms per-snapshot gradients and weights them by the snapshot's upstream gradient).  The
    forward of energies(..., "bf16"); gz2 = q(W2 silu'(z2)); gh1 = q(W1)^T gz2;
    gz1 = q(gh1 silu'(z1)); dW1 = sum g gz2 (x) q(h1) (h1 as the forward feeds layer 1);
    dW0, db0 = sum g gz1 (x) x; db1 = sum g gz2; dW2 = sum g silu(z2); db2 = sum g; q = BF16."""
    W0, b0, W1, b1, W2, b2 = split_params(params)
    X = np.asarray(X, dtype=np.float64)
    g = np.asarray(g_rows, dtype=np.float64)[:, None]
    f64 = np.float64
    W0s = (-L2E * W0).astype(np.float32)
    c0 = (-L2E * b0).astype(np.float32)
    c1 = (-L2E * b1).astype(np.float32)
    y1 = (X @ bf16(W0s).T.astype(f64) + bf16(c0)).astype(np.float32)
    a1 = bf16(act(y1))                                   # -log2(e) h1, as staged
    y2 = (a1.astype(f64) @ bf16(W1).T.astype(f64) + c1).astype(np.float32)
    z2 = (-LN2 * y2).astype(np.float32)
    sg2 = (np.float32(1.0) / (np.float32(1.0) + np.exp2(y2))).astype(np.float32)
    gz2 = bf16((W2.astype(np.float32)[None, :] * dsilu_from_y(y2)).astype(np.float32))
    hg = g * (z2 * sg2).astype(np.float64)
    gh1 = (gz2.astype(f64) @ bf16(W1).astype(f64)).astype(np.float32)
    gz1 = g * bf16((gh1 * dsilu_from_y(y1)).astype(np.float32)).astype(f64)
    gz2 = g * gz2.astype(f64)
    dW1 = -np.float64(LN2) * (gz2.T @ a1.astype(f64))
    dW0 = gz1.T @ X
    out = np.concatenate([dW0.ravel(), gz1.sum(axis=0), dW1.ravel(), gz2.sum(axis=0), hg.sum(axis=0), [g.sum()]])
    return out


def snapshot_rows(cells, snaps):
    """One-hot feature rows [batch * N, 108] of every site of every snapshot (oracle features)."""
    import oracle
    rows = []
    for s in snaps:
        for j in range(s.size):
            rows.append(oracle.features(cells, 1, s, j))
    return np.asarray(rows)


def _mlpnet_fp8(W0, b0, W1, b1, W2, b2, W3, b3, X, n_slots=19):
    """FP8 MLPNet as the FCC evaluator defines it: E4M3 weights W / 2^k per layer (the largest
    |W| at most 448); the activation entering layer l + 1 is E4M3(relu(z_l) / 2^kh_l), with
    kh_l from the bound hmax_0 = max_u (b0 + sum over slots of the largest positive weight),
    hmax_1 = max_u (b1 + sum_k max(W1, 0) hmax_0); every bias starts its FP32 accumulator."""
    p2 = _pow2_at_least
    W0d, W1d, W2d = (W.astype(np.float64) for W in (W0, W1, W2))
    k0, k1, k2 = (p2(float(np.abs(W).max()) / 448.0) for W in (W0, W1, W2))
    H = W0.shape[0]
    z = b0.astype(np.float64) + np.maximum(0.0, W0d.reshape(H, n_slots, 4).max(axis=2)).sum(axis=1)
    h0 = max(0.0, float(z.max()))
    z = b1.astype(np.float64) + np.maximum(0.0, W1d).sum(axis=1) * h0
    h1 = max(0.0, float(z.max()))
    kh0, kh1 = p2(h0 / 448.0), p2(h1 / 448.0)
    A0 = e4m3(W0 * np.float32(2.0 ** -k0)).astype(np.float64) * 2.0 ** k0
    A1 = e4m3(W1 * np.float32(2.0 ** -k1)).astype(np.float64) * 2.0 ** k1
    A2 = e4m3(W2 * np.float32(2.0 ** -k2)).astype(np.float64) * 2.0 ** k2
    # layers 0 and 1 accumulate in units of the next activation scale
    z0 = ((b0 * np.float32(2.0 ** -kh0)).astype(np.float64) + (X @ A0.T) * 2.0 ** -kh0).astype(np.float32)
    a1 = e4m3(np.maximum(z0, 0)).astype(np.float64)
    z1 = ((b1 * np.float32(2.0 ** -kh1)).astype(np.float64) + (a1 @ A1.T) * 2.0 ** (kh0 - kh1)).astype(np.float32)
    a2 = e4m3(np.maximum(z1, 0)).astype(np.float64)
    z2 = (b2.astype(np.float64) + (a2 @ A2.T) * 2.0 ** kh1).astype(np.float32)
    return np.maximum(z2, 0).astype(np.float64) @ W3.astype(np.float64) + float(b3)


def mlpnet_emulate(params, X, prec, H=96, n_in=76):
    """MLPNet (Eqs. (4)-(6)) as the FCC matrix-core evaluator computes it: layer 0 takes the
    bias as a weight column on a constant-one input, later biases start the FP32 accumulators,
    ReLU, W3 and b3 in FP32; q() quantises weights and the activations entering layers 1 and 2
    (bf16x3: hi*hi + hi*lo + lo*hi; fp8: see _mlpnet_fp8).  X: [rows][76] one-hot features
    (exact in every format)."""
    p = np.asarray(params, dtype=np.float32)
    o = 0
    W0 = p[o:o + H * n_in].reshape(H, n_in); o += H * n_in
    b0 = p[o:o + H]; o += H
    W1 = p[o:o + H * H].reshape(H, H); o += H * H
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + H]; o += H
    b3 = p[o]
    X = np.asarray(X, dtype=np.float64)
    if prec == "fp8":
        return _mlpnet_fp8(W0, b0, W1, b1, W2, b2, W3, b3, X)

    def split(a):
        hi = bf16(a)
        return hi.astype(np.float64), bf16(a - hi).astype(np.float64)

    def matmul(Wm, A):  # Wm [out][in] fp32, A [rows][in] fp32 activations
        if prec == "fp32":
            return A.astype(np.float64) @ Wm.astype(np.float64).T
        wh, wl = split(Wm)
        ah, al = split(A)
        if prec == "bf16":
            return ah @ wh.T
        return ah @ wh.T + al @ wh.T + ah @ wl.T

    W0b = np.concatenate([W0, b0[:, None]], axis=1)
    Xb = np.concatenate([X, np.ones((X.shape[0], 1))], axis=1).astype(np.float32)
    z1 = matmul(W0b, Xb).astype(np.float32)
    h1 = np.maximum(z1, 0).astype(np.float32)
    z2 = (matmul(W1, h1) + b1).astype(np.float32)
    h2 = np.maximum(z2, 0).astype(np.float32)
    z3 = (matmul(W2, h2) + b2).astype(np.float32)
    h3 = np.maximum(z3, 0).astype(np.float64)
    return h3 @ W3.astype(np.float64) + float(b3)
