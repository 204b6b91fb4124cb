"""FP64 reference of the warm-start surrogate's convolutions (numpy).

TEST INFRASTRUCTURE ONLY.  Plain definitions, one tap at a time:

  forward          y[s,co,v] = b[co] + sum_{tap,ci} w[co,tap,ci] xpad[s,ci,v + d_tap]
  backward data    dx[s,ci,v] = sum_{tap,co} w[co,tap,ci] dypad[s,co,v - d_tap]
  backward weight  dw[co,tap,ci] = sum_{s,v} dy[s,co,v] xpad[s,ci,v + d_tap],
                   db[co] = sum_{s,v} dy[s,co,v]

Arrays are [sample][channel][z][y][x] without halo; x and y are periodic;
z is padded with a constant per input channel (`zpad`, the wall value).
tap = (dz+1)*9 + (dy+1)*3 + (dx+1).
"""
from __future__ import annotations

import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def _shift(a, dz, dy, dx, zpad):
    """a[..., z + dz, y + dy, x + dx] with periodic x, y and constant z padding
    (zpad: one value per channel, axis 1)."""
    s, c, nz, ny, nx = a.shape
    out = np.roll(np.roll(a, -dy, axis=3), -dx, axis=4)
    if dz == 0:
        return out
    pad = np.broadcast_to(np.asarray(zpad, dtype=np.float64).reshape(1, c, 1, 1, 1), (s, c, 1, ny, nx))
    if dz == 1:
        return np.concatenate([out[:, :, 1:], pad], axis=2)
    return np.concatenate([pad, out[:, :, :-1]], axis=2)


def conv_forward(x, w, b, zpad=None, relu=False):
    """x [S,Cin,Z,Y,X], w [Cout,27,Cin], b [Cout] -> [S,Cout,Z,Y,X]."""
    x = np.asarray(x, dtype=np.float64)
    cin = x.shape[1]
    zpad = np.zeros(cin) if zpad is None else zpad
    y = np.zeros((x.shape[0], w.shape[0]) + x.shape[2:])
    for t, (dz, dy, dx) in enumerate(TAPS):
        y += np.einsum("oc,sczyx->sozyx", w[:, t, :], _shift(x, dz, dy, dx, zpad))
    y += np.asarray(b, dtype=np.float64).reshape(1, -1, 1, 1, 1)
    return np.maximum(y, 0.0) if relu else y


def conv_backward_data(dy, w):
    """dy [S,Cout,Z,Y,X], w [Cout,27,Cin] -> dx [S,Cin,Z,Y,X] (zero outside z)."""
    cout = dy.shape[1]
    dx = np.zeros((dy.shape[0], w.shape[2]) + dy.shape[2:])
    for t, (dz, dy_, dx_) in enumerate(TAPS):
        dx += np.einsum("oc,sozyx->sczyx", w[:, t, :], _shift(dy, -dz, -dy_, -dx_, np.zeros(cout)))
    return dx


def conv_backward_weight(x, dy, zpad=None):
    """x [S,Cin,Z,Y,X], dy [S,Cout,Z,Y,X] -> dw [Cout,27,Cin], db [Cout]."""
    cin = x.shape[1]
    zpad = np.zeros(cin) if zpad is None else zpad
    dw = np.zeros((dy.shape[1], 27, cin))
    for t, (dz, dy_, dx_) in enumerate(TAPS):
        dw[:, t, :] = np.einsum("sozyx,sczyx->oc", dy, _shift(x, dz, dy_, dx_, zpad))
    return dw, dy.sum(axis=(0, 2, 3, 4))


def bf16_round(a):
    """Round to the nearest bfloat16 (8 significand bits, ties to even), via
    float32: the value's float32 bit pattern has its low 16 bits rounded
    away.  Returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def network_forward(x0, layers, zpad0, store=None):
    """layers: list of (w, b, relu); returns all activations (input first).
    store, if given, is applied to every hidden activation as it is kept (the
    output layer's values are not)."""
    acts = [np.asarray(x0, dtype=np.float64)]
    for i, (w, b, relu) in enumerate(layers):
        zp = zpad0 if i == 0 else None
        y = conv_forward(acts[-1], w, b, zp, relu)
        acts.append(store(y) if (store is not None and i < len(layers) - 1) else y)
    return acts


def network_loss_and_grads(x0, layers, zpad0, target, store=None):
    """MSE = mean over samples, 3 channels and voxels of (y - target)^2, and
    its gradient with respect to every weight and bias.  store, if given, is
    applied to every kept hidden activation and to every activation gradient
    (the output gradient, and each backward-data result after its ReLU
    mask), the points where a network keeping those in a narrower format
    rounds them."""
    acts = network_forward(x0, layers, zpad0, store)
    out = acts[-1]
    n = out.size
    loss = float(((out - target) ** 2).sum() / n)
    g = 2.0 * (out - target) / n
    grads = [None] * len(layers)
    for i in range(len(layers) - 1, -1, -1):
        w, b, relu = layers[i]
        if relu:
            g = g * (acts[i + 1] > 0)
        if store is not None:
            g = store(g)
        zp = zpad0 if i == 0 else None
        grads[i] = conv_backward_weight(acts[i], g, zp)
        if i > 0:
            g = conv_backward_data(g, w)
    return loss, grads
