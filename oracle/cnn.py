"""Oracle: the learned MB localiser (FP64, CPU).

TEST INFRASTRUCTURE ONLY.

The paper names deep-learning localisation as a way to go beyond NCC
(Section IV).  The learned form here is a small 2D CNN on the filtered
projection envelope:
  input   I / max_frame(I), one channel, H x W (the plane grid)
  layers  conv3x3 (1 -> C) + ReLU, then L-1 x conv3x3 (C -> C) + ReLU,
          zero padding 1, C = 32, L = 6
  head    1x1 conv (C -> R^2) and depth-to-space with factor R = 8: a heatmap
          on a grid R times finer than the plane
  target  T(q) = max over MBs of exp(-|q - R (x + 1/2) + 1/2|^2 / (2 s^2)), s = 1
          fine pixel, x the MB position in plane pixel units (centres at
          integers), q the fine pixel index
  loss    mean squared error over the fine grid
  update  Adam (Kingma and Ba, 2015)
Tensors are channel-first: activations [C][H][W], conv weights [out][in][3][3].
"""
from __future__ import annotations

import numpy as np

R = 8


def init_params(rng, channels=32, layers=6, r=R):
    """He-normal conv weights, zero biases; head small normal."""
    p = {}
    cin = 1
    for l in range(layers):
        std = np.sqrt(2.0 / (9 * cin))
        p[f"w{l}"] = rng.standard_normal((channels, cin, 3, 3)) * std
        p[f"b{l}"] = np.zeros(channels)
        cin = channels
    p["wh"] = rng.standard_normal((r * r, channels)) * np.sqrt(1.0 / channels)
    p["bh"] = np.zeros(r * r)
    return p


def conv3x3(x, w, b):
    """y[o] = b[o] + sum_c sum_{dy,dx} w[o,c,dy,dx] x[c, i+dy-1, j+dx-1] (zero padding)."""
    C, H, W = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1)))
    y = np.broadcast_to(b[:, None, None], (w.shape[0], H, W)).copy()
    for dy in range(3):
        for dx in range(3):
            y += np.einsum("oc,chw->ohw", w[:, :, dy, dx], xp[:, dy:dy + H, dx:dx + W])
    return y


def conv3x3_backward(x, w, gy):
    """Gradients of conv3x3 w.r.t. its input, weights and bias."""
    C, H, W = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1)))
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w)
    for dy in range(3):
        for dx in range(3):
            gw[:, :, dy, dx] = np.einsum("ohw,chw->oc", gy, xp[:, dy:dy + H, dx:dx + W])
            gxp[:, dy:dy + H, dx:dx + W] += np.einsum("oc,ohw->chw", w[:, :, dy, dx], gy)
    return gxp[:, 1:-1, 1:-1], gw, gy.sum(axis=(1, 2))


def depth_to_space(y, r=R):
    """[r*r][H][W] -> [H*r][W*r]: out[h*r + i, w*r + j] = y[i*r + j, h, w]."""
    rr, H, W = y.shape
    return y.reshape(r, r, H, W).transpose(2, 0, 3, 1).reshape(H * r, W * r)


def space_to_depth(z, r=R):
    Hr, Wr = z.shape
    return z.reshape(Hr // r, r, Wr // r, r).transpose(1, 3, 0, 2).reshape(r * r, Hr // r, Wr // r)


def forward(p, img, layers=6):
    """Returns (heatmap [H*R][W*R], cache)."""
    acts = [img[None, :, :]]
    pre = []
    x = acts[0]
    for l in range(layers):
        z = conv3x3(x, p[f"w{l}"], p[f"b{l}"])
        pre.append(z)
        x = np.maximum(z, 0.0)
        acts.append(x)
    h = np.einsum("kc,chw->khw", p["wh"], x) + p["bh"][:, None, None]
    return depth_to_space(h), (acts, pre)


def target_map(positions, H, W, r=R, s=1.0):
    """T(q) = max_MB exp(-|q - (r (x + 1/2) - 1/2)|^2 / (2 s^2)) on the fine grid.
    positions: [n][2] (z, u) in plane pixel units."""
    T = np.zeros((H * r, W * r))
    if len(positions) == 0:
        return T
    rad = int(np.ceil(4 * s))
    for (z, u) in positions:
        cz, cu = r * (z + 0.5) - 0.5, r * (u + 0.5) - 0.5
        z0, z1 = max(0, int(np.floor(cz)) - rad), min(H * r, int(np.floor(cz)) + rad + 2)
        u0, u1 = max(0, int(np.floor(cu)) - rad), min(W * r, int(np.floor(cu)) + rad + 2)
        if z0 >= z1 or u0 >= u1:
            continue
        qz, qu = np.meshgrid(np.arange(z0, z1), np.arange(u0, u1), indexing="ij")
        g = np.exp(-((qz - cz) ** 2 + (qu - cu) ** 2) / (2 * s * s))
        T[z0:z1, u0:u1] = np.maximum(T[z0:z1, u0:u1], g)
    return T


def loss_and_grad(p, img, T, layers=6):
    """MSE loss and gradients of every parameter."""
    hm, (acts, pre) = forward(p, img, layers)
    n = hm.size
    diff = hm - T
    loss = float(np.mean(diff * diff))
    g_hm = 2.0 * diff / n
    gh = space_to_depth(g_hm)                        # [r*r][H][W]
    x = acts[-1]
    grads = {"wh": np.einsum("khw,chw->kc", gh, x), "bh": gh.sum(axis=(1, 2))}
    gx = np.einsum("kc,khw->chw", p["wh"], gh)
    for l in reversed(range(layers)):
        gz = gx * (pre[l] > 0)
        gx, gw, gb = conv3x3_backward(acts[l], p[f"w{l}"], gz)
        grads[f"w{l}"], grads[f"b{l}"] = gw, gb
    return loss, grads


def adam_step(p, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in place; state holds m, v and the step count t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in p:
        m = state.setdefault("m_" + k, np.zeros_like(p[k]))
        v = state.setdefault("v_" + k, np.zeros_like(p[k]))
        m[...] = b1 * m + (1 - b1) * grads[k]
        v[...] = b2 * v + (1 - b2) * grads[k] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p


def decode(hm, thresh=0.5, r=R):
    """Local maxima (3x3, raster tie-break) of the heatmap at or above `thresh`;
    positions in plane pixel units."""
    Hr, Wr = hm.shape
    pad = np.full((Hr + 2, Wr + 2), -np.inf)
    pad[1:-1, 1:-1] = hm
    c = hm >= thresh
    for dz, du in [(-1, -1), (-1, 0), (-1, 1), (0, -1)]:
        c &= hm > pad[1 + dz:1 + dz + Hr, 1 + du:1 + du + Wr]
    for dz, du in [(0, 1), (1, -1), (1, 0), (1, 1)]:
        c &= hm >= pad[1 + dz:1 + dz + Hr, 1 + du:1 + du + Wr]
    qz, qu = np.nonzero(c)
    return np.stack([(qz + 0.5) / r - 0.5, (qu + 0.5) / r - 0.5], axis=1) if qz.size else \
        np.zeros((0, 2))
