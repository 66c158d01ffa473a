"""FP64 reference of the yield surrogate MLP (forward, loss, gradient).

TEST INFRASTRUCTURE ONLY: used to check the GPU surrogate kernels.  Plain
numpy in float64, written from the definition of the network:

    h_0 = x;  z_l = W_l h_{l-1} + b_l;  h_l = GELU(z_l)  (l = 1..depth)
    y = w_out . h_depth + b_out;  loss = mean over the batch of (y - t)^2

GELU(z) = z Phi(z) with the standard normal CDF Phi; its derivative is
Phi(z) + z phi(z).  Gradients are the chain rule written out layer by layer.
Parameter vector order: W_1 (rows = output units), b_1, ..., W_depth,
b_depth, w_out, b_out.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_d(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def unpack(params, n_in, width=256, depth=4):
    p = np.asarray(params, dtype=np.float64)
    o = 0
    Ws, bs = [], []
    for l in range(depth):
        kin = n_in if l == 0 else width
        Ws.append(p[o:o + width * kin].reshape(width, kin))
        o += width * kin
        bs.append(p[o:o + width])
        o += width
    w_out = p[o:o + width]
    o += width
    b_out = p[o]
    o += 1
    assert o == p.size
    return Ws, bs, w_out, b_out


def n_params(n_in, width=256, depth=4):
    return width * n_in + width + (depth - 1) * (width * width + width) + width + 1


def forward(params, X, n_in, width=256, depth=4):
    Ws, bs, w_out, b_out = unpack(params, n_in, width, depth)
    h = np.asarray(X, dtype=np.float64)
    zs, hs = [], [h]
    for W, b in zip(Ws, bs):
        z = h @ W.T + b
        h = gelu(z)
        zs.append(z)
        hs.append(h)
    y = h @ w_out + b_out
    return y, (zs, hs)


def loss_and_grad(params, X, t, n_in, width=256, depth=4):
    Ws, bs, w_out, b_out = unpack(params, n_in, width, depth)
    y, (zs, hs) = forward(params, X, n_in, width, depth)
    t = np.asarray(t, dtype=np.float64)
    B = y.shape[0]
    loss = float(np.mean((y - t) ** 2))
    dy = 2.0 * (y - t) / B
    g_wout = hs[-1].T @ dy
    g_bout = dy.sum()
    dh = np.outer(dy, w_out)
    gW = [None] * depth
    gb = [None] * depth
    for l in range(depth - 1, -1, -1):
        dz = dh * gelu_d(zs[l])
        gW[l] = dz.T @ hs[l]
        gb[l] = dz.sum(axis=0)
        dh = dz @ Ws[l]
    parts = []
    for l in range(depth):
        parts.append(gW[l].ravel())
        parts.append(gb[l])
    parts.append(g_wout)
    parts.append(np.array([g_bout]))
    return loss, np.concatenate(parts)


def round_bf16(a):
    """Round float32 values to the nearest bfloat16 (ties to even), back as float32."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).reshape(a.shape)


def gpu_visible_params(params, n_in, width=256, depth=4):
    """Parameters as the GPU multiplies them: weight matrices rounded to bfloat16;
    biases and the output layer kept in FP32."""
    p = np.asarray(params, dtype=np.float32).copy()
    o = 0
    for l in range(depth):
        kin = n_in if l == 0 else width
        p[o:o + width * kin] = round_bf16(p[o:o + width * kin])
        o += width * kin + width
    return p
