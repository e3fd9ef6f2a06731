"""ORACLE -- test infrastructure only (tests/, the smoke check and the
benchmark's CPU leg load it; the GPU path never does).

Plain NumPy float64 reference of the learned coarse-flow proposal: a 6-layer
3x3 convolutional network that maps the stacked RGB pair to a 2-channel flow
on the 1/8 grid (the seed grid of a 3-level hierarchy), evaluated as one
extra seed candidate (the exact data term still decides every match).

Architecture (fixed): (Cin, Cout, stride, dilation, ReLU)
    L1 (6, 32, 2, 1, yes)  L2 (32, 32, 2, 1, yes)  L3 (32, 32, 2, 1, yes)
    L4 (32, 32, 1, 4, yes) L5 (32, 32, 1, 8, yes)  L6 (32, 2, 1, 1, no)
padding = dilation ("same" for stride 1, ceil(H/2) for stride 2); the
receptive field is about 220 px.  Input x = RGB/255 - 1/2 for both frames;
output flow in pixels = 32 * L6.

Precision: weights and stored activations are bfloat16 (round to nearest
even), every product sum is accumulated in float64 here (float32 on the
GPU); back-propagated activation gradients are stored in bfloat16 as well.
`exact=True` turns all rounding off (used by the finite-difference pins).

Parameter layout: for each layer W[co][ci][ky][kx] then b[co], float32.
"""
from __future__ import annotations

import numpy as np

LAYERS = [(6, 32, 2, 1, True), (32, 32, 2, 1, True), (32, 32, 2, 1, True),
          (32, 32, 1, 4, True), (32, 32, 1, 8, True), (32, 2, 1, 1, False)]
FLOW_SCALE = 32.0


def param_count() -> int:
    return sum(co * ci * 9 + co for ci, co, _, _, _ in LAYERS)


def split_params(theta):
    out = []
    o = 0
    for ci, co, _, _, _ in LAYERS:
        W = theta[o:o + co * ci * 9].reshape(co, ci, 3, 3)
        o += co * ci * 9
        b = theta[o:o + co]
        o += co
        out.append((W, b))
    return out


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights, zero biases (float32)."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co, _, _, relu in LAYERS:
        std = np.sqrt(2.0 / (ci * 9)) if relu else np.sqrt(1.0 / (ci * 9))
        parts.append((rng.standard_normal(co * ci * 9) * std).astype(np.float32))
        parts.append(np.zeros(co, np.float32))
    return np.concatenate(parts)


def bf16(x, exact=False):
    """Round to bfloat16 (nearest even), returned as float64."""
    if exact:
        return np.asarray(x, np.float64)
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def out_size(n, stride):
    return (n + stride - 1) // stride


def conv(x, W, b, stride, dil):
    """x: B x H x W x Ci, W: Co x Ci x 3 x 3 -> B x Ho x Wo x Co (float64),
    zero padding = dil."""
    B, H, Wd, Ci = x.shape
    Co = W.shape[0]
    Ho, Wo = out_size(H, stride), out_size(Wd, stride)
    p = dil
    xp = np.zeros((B, H + 2 * p + 2 * dil, Wd + 2 * p + 2 * dil, Ci), np.float64)
    xp[:, p:p + H, p:p + Wd] = x
    y = np.zeros((B, Ho, Wo, Co), np.float64)
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky * dil: ky * dil + stride * (Ho - 1) + 1: stride,
                       kx * dil: kx * dil + stride * (Wo - 1) + 1: stride, :]
            y += patch @ W[:, :, ky, kx].T.astype(np.float64)
    return y + b.astype(np.float64)


def conv_backward(x, W, gy, stride, dil):
    """Gradients of conv(x, W, b) given dL/dy: (dx, dW, db)."""
    B, H, Wd, Ci = x.shape
    Co = W.shape[0]
    Ho, Wo = gy.shape[1:3]
    p = dil
    xp = np.zeros((B, H + 2 * p + 2 * dil, Wd + 2 * p + 2 * dil, Ci), np.float64)
    xp[:, p:p + H, p:p + Wd] = x
    gxp = np.zeros_like(xp)
    dW = np.zeros(W.shape, np.float64)
    for ky in range(3):
        for kx in range(3):
            sl = (slice(None), slice(ky * dil, ky * dil + stride * (Ho - 1) + 1, stride),
                  slice(kx * dil, kx * dil + stride * (Wo - 1) + 1, stride), slice(None))
            patch = xp[sl]
            dW[:, :, ky, kx] = np.einsum("bhwc,bhwo->oc", patch, gy)
            gxp[sl] += gy @ W[:, :, ky, kx].astype(np.float64)
    db = gy.sum(axis=(0, 1, 2))
    return gxp[:, p:p + H, p:p + Wd], dW, db


def input_tensor(img1, img2, exact=False):
    """Stack two H x W x 3 uint8 frames (or B x H x W x 3) into B x H x W x 6."""
    a = np.asarray(img1, np.float64)
    c = np.asarray(img2, np.float64)
    if a.ndim == 3:
        a, c = a[None], c[None]
    x = np.concatenate([a, c], -1) / 255.0 - 0.5
    return bf16(x, exact)


def forward(theta, x, exact=False, keep=False):
    """Returns the L6 output (B x Hc x Wc x 2, float64; flow px = 32 * out)
    and, with keep=True, the list of layer inputs/outputs for backward."""
    acts = [x]
    a = x
    for (ci, co, s, d, relu), (W, b) in zip(LAYERS, split_params(theta)):
        z = conv(a, bf16(W, exact), b, s, d)
        if relu:
            a = bf16(np.maximum(z, 0.0), exact)
        else:
            a = z
        acts.append(a)
    return (a, acts) if keep else a


def masked_l1(out, labels_px):
    """Mean over labelled grid points of |dx| + |dy| in output units (px/32);
    labels_px: B x Hc x Wc x 2 float with NaN where there is no label."""
    mask = ~np.isnan(labels_px[..., 0])
    n = max(int(mask.sum()), 1)
    t = np.nan_to_num(labels_px) / FLOW_SCALE
    diff = (out - t) * mask[..., None]
    loss = np.abs(diff).sum() / n
    grad = np.sign(diff) * mask[..., None] / n
    return loss, grad


def backward(theta, acts, gout, exact=False, magnitude=False):
    """Parameter gradient (float64, parameter layout) from dL/d(out).  With
    magnitude=True also the gradient's magnitude in the same layout: each
    weight's sum of |input activation| x |output gradient| over its products
    and each bias's sum of |output gradient| (the scale of the rounding
    error a sum of those products can carry)."""
    params = split_params(theta)
    grads = [None] * len(LAYERS)
    mags = [None] * len(LAYERS)
    g = gout
    for li in range(len(LAYERS) - 1, -1, -1):
        ci, co, s, d, relu = LAYERS[li]
        W, b = params[li]
        if relu:
            g = bf16(g * (acts[li + 1] > 0), exact)
        else:
            g = bf16(g, exact)
        gx, dW, db = conv_backward(acts[li], bf16(W, exact), g, s, d)
        grads[li] = (dW, db)
        if magnitude:
            _, mW, mb = conv_backward(np.abs(acts[li]), np.abs(bf16(W, exact)), np.abs(g), s, d)
            mags[li] = (mW, mb)
        g = gx
    flat = np.concatenate([np.concatenate([dW.reshape(-1), db]) for dW, db in grads])
    if not magnitude:
        return flat
    return flat, np.concatenate([np.concatenate([mW.reshape(-1), mb]) for mW, mb in mags])


def forward_magnitude(theta, acts):
    """Per output element of the last layer, the sum of |weight| x |input
    activation| over its products plus |bias| (the scale of the rounding
    error the last layer's sum can carry)."""
    (ci, co, s, d, relu), (W, b) = LAYERS[-1], split_params(theta)[-1]
    return conv(np.abs(acts[-2]), np.abs(bf16(W)), np.abs(b), s, d)


def adam_step(theta, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def proposal_q(out, subpel=4):
    """Round the network's flow to packed int16x2 (1/Q px), nearest even."""
    fx = np.clip(np.rint(out[..., 0] * FLOW_SCALE * subpel), -32767, 32767).astype(np.int64)
    fy = np.clip(np.rint(out[..., 1] * FLOW_SCALE * subpel), -32767, 32767).astype(np.int64)
    v = ((fy & 0xFFFF) << 16) | (fx & 0xFFFF)
    return np.where(v >= 1 << 31, v - (1 << 32), v).astype(np.int32)
