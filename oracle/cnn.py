"""CPU oracle of the candidate-pruning network -- TEST INFRASTRUCTURE ONLY.

A 3-layer 3x3 convolutional network, 4 -> 16 -> 16 -> 1 channels, ReLU after the first two
layers, zero padding, scored per pixel with a weighted binary cross-entropy.  Everything is
FP64 written out from the definitions; where the GPU stores a tensor in BF16 (weights,
inputs, activations, back-propagated errors) the oracle rounds that tensor to BF16
(round to nearest even) at the same point, so the GPU result must agree up to FP32
accumulation order.  Only tests, the smoke check and the benchmark's CPU leg may import it.

Layout: activations [H, W, C], weights [3, 3, Cin, Cout] (row offset, column offset,
input channel, output channel), biases [Cout].
"""
from __future__ import annotations

import numpy as np

C_IN, C_HID = 4, 16


def bf16(x):
    """Round to the nearest BF16 value, ties to even, returned as FP64."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    nan = np.isnan(a)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(nan, np.nan, out)


# ----------------------------------------------------------------------------- features
def sobel(grey):
    """G_x, G_y with weights (1,2,1), zero outside the image (the lane detector's Sobel)."""
    g = np.pad(grey.astype(np.float64), 1)
    gx = (g[:-2, 2:] - g[:-2, :-2]) + 2 * (g[1:-1, 2:] - g[1:-1, :-2]) + (g[2:, 2:] - g[2:, :-2])
    gy = (g[2:, :-2] - g[:-2, :-2]) + 2 * (g[2:, 1:-1] - g[:-2, 1:-1]) + (g[2:, 2:] - g[:-2, 2:])
    return gx, gy


def features(grey, disp_values, valid, f_rows, varpi=3.0):
    """Four input channels per pixel of a band of rows:
    intensity I/255; gradient magnitude sqrt(G_x^2 + G_y^2)/1020; gradient direction
    atan2(G_y, G_x)/pi; disparity residual to the road profile clamp((D - f(v))/varpi, -4, 4)
    (-4 where the disparity is invalid).  grey: [H, W] of the band plus one row above and
    below (Sobel support); disp_values/valid: [H-2, W]; f_rows: [H-2]."""
    gx, gy = sobel(grey)
    gx, gy = gx[1:-1], gy[1:-1]
    inner = grey[1:-1].astype(np.float64)
    res = np.clip((disp_values - f_rows[:, None]) / varpi, -4.0, 4.0)
    res = np.where(valid, res, -4.0)
    return np.stack([inner / 255.0, np.sqrt(gx * gx + gy * gy) / 1020.0, np.arctan2(gy, gx) / np.pi, res], axis=-1)


# ----------------------------------------------------------------------------- network
def conv3x3(x, w, b):
    """y[v,u,o] = b[o] + sum_{i,j,c} x[v+i-1, u+j-1, c] w[i,j,c,o], zero padding."""
    H, W, _ = x.shape
    xp = np.pad(x, ((1, 1), (1, 1), (0, 0)))
    y = np.zeros((H, W, w.shape[3])) + b
    for i in range(3):
        for j in range(3):
            y += xp[i:i + H, j:j + W, :] @ w[i, j]
    return y


def init_params(seed=0):
    rng = np.random.default_rng(seed)
    p = {}
    for name, (ci, co) in {"1": (C_IN, C_HID), "2": (C_HID, C_HID), "3": (C_HID, 1)}.items():
        p["w" + name] = bf16(rng.normal(0.0, np.sqrt(2.0 / (9 * ci)), size=(3, 3, ci, co)))
        p["b" + name] = np.zeros(co)
    p["b3"] = np.full(1, -2.0)
    return p


def forward(x, p, emulate_bf16=True):
    """Returns (z1, a1, z2, a2, z3): pre-activations z, activations a, logits z3 [H, W, 1]."""
    r = bf16 if emulate_bf16 else (lambda t: t)
    x = r(x)
    z1 = conv3x3(x, r(p["w1"]), p["b1"])
    a1 = r(np.maximum(z1, 0.0))
    z2 = conv3x3(a1, r(p["w2"]), p["b2"])
    a2 = r(np.maximum(z2, 0.0))
    z3 = conv3x3(a2, r(p["w3"]), p["b3"])
    return z1, a1, z2, a2, z3


def softplus(z):
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def loss_and_grad_logits(z3, label, mask, pos_weight):
    """Weighted BCE with logits, averaged over the masked pixels:
    l = pw*y*softplus(-z) + (1-y)*softplus(z); dl/dz = pw*y*(sigmoid(z)-1) + (1-y)*sigmoid(z)."""
    z = z3[..., 0]
    n = max(1.0, float(mask.sum()))
    l = pos_weight * label * softplus(-z) + (1 - label) * softplus(z)
    g = pos_weight * label * (sigmoid(z) - 1.0) + (1 - label) * sigmoid(z)
    return float((l * mask).sum() / n), (g * mask / n)[..., None]


def conv3x3_backward(x, w, dy):
    """Gradients of y = conv3x3(x, w, b) given dy: (dx, dw, db)."""
    H, W, _ = x.shape
    xp = np.pad(x, ((1, 1), (1, 1), (0, 0)))
    dw = np.zeros_like(w)
    for i in range(3):
        for j in range(3):
            dw[i, j] = xp[i:i + H, j:j + W, :].reshape(-1, x.shape[2]).T @ dy.reshape(-1, dy.shape[2])
    db = dy.sum(axis=(0, 1))
    dyp = np.pad(dy, ((1, 1), (1, 1), (0, 0)))
    dx = np.zeros_like(x)
    for i in range(3):
        for j in range(3):
            # x[v, u] feeds y[v - i + 1, u - j + 1] through w[i, j]
            dx += dyp[2 - i:2 - i + H, 2 - j:2 - j + W, :] @ w[i, j].T
    return dx, dw, db


def backward(x, p, cache, dz3, emulate_bf16=True):
    """Parameter gradients of the network for the logit gradient dz3 (chain rule)."""
    r = bf16 if emulate_bf16 else (lambda t: t)
    z1, a1, z2, a2, _ = cache
    dz3 = r(dz3)
    da2, dw3, db3 = conv3x3_backward(a2, r(p["w3"]), dz3)
    dz2 = r(da2 * (z2 > 0))
    da1, dw2, db2 = conv3x3_backward(a1, r(p["w2"]), dz2)
    dz1 = r(da1 * (z1 > 0))
    _, dw1, db1 = conv3x3_backward(r(x), r(p["w1"]), dz1)
    return {"w1": dw1, "b1": db1, "w2": dw2, "b2": db2, "w3": dw3, "b3": db3}


def adam_step(p, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update of FP64 master weights (the GPU keeps FP32 masters)."""
    out = {}
    for k in p:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] * g[k]
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        out[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return out


# ----------------------------------------------------------------------------- glue
ORDER = [("w1", (3, 3, C_IN, C_HID)), ("b1", (C_HID,)), ("w2", (3, 3, C_HID, C_HID)), ("b2", (C_HID,)),
         ("w3", (3, 3, C_HID, 1)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in ORDER)


def flat(p):
    """Parameters as one vector in the library's order: w1, b1, w2, b2, w3, b3 (row-major)."""
    return np.concatenate([np.asarray(p[k], np.float64).reshape(-1) for k, _ in ORDER])


def unflat(v):
    out, o = {}, 0
    for k, s in ORDER:
        n = int(np.prod(s))
        out[k] = np.asarray(v[o:o + n], np.float64).reshape(s)
        o += n
    return out


def disparity_values(disp):
    """D and validity per pixel: u8 raw (0 invalid), f32 raw (finite and > 0), u16 raw / 16 (0 invalid)."""
    if disp.dtype == np.uint8:
        return disp.astype(np.float64), disp != 0
    if disp.dtype == np.float32:
        ok = np.isfinite(disp) & (disp > 0)
        return np.where(ok, disp, 0).astype(np.float64), ok
    return disp.astype(np.float64) / 16.0, disp != 0


def band_top(v_h, H, n_bands, k):
    """First row of band k (0 = bottom) of 16 road rows, or -1 when the road has fewer than 16 rows."""
    R = H - v_h
    if R < 16 or n_bands < 1:
        return -1
    return (H - 16) - ((R - 16) * k) // n_bands


def band_features(grey, disp, f_table, top, varpi=3.0):
    """The network input of the 16-row band starting at `top` of a frame: [16, W, 4]."""
    H, W = grey.shape
    g = np.zeros((18, W), np.float64)
    lo, hi = max(top - 1, 0), min(top + 17, H)
    g[lo - (top - 1):hi - (top - 1)] = grey[lo:hi]
    D, ok = disparity_values(disp[top:top + 16])
    return features(g, D, ok, np.asarray(f_table)[top:top + 16], varpi)
