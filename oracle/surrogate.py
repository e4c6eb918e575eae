"""The learned surrogate of the grid convolution, written plainly (FP64 numpy).

Test infrastructure, like the rest of ``oracle/``. The surrogate replaces
step 2 of the AIM (Sec. 3.2.2: the FFT convolution of the grid charges Q with
the periodic Green's function, giving the grid potential U) by a network of
3x3x3 convolution layers. This module holds the definitions that the
library's hand-written kernels must reproduce:

* a layer: out[co, z, y, x] = b[co] + sum_ci sum_(dz,dy,dx in -1..1)
  W[co, ci, dz+1, dy+1, dx+1] in[ci, z+dz, (y+dy) mod Ny, (x+dx) mod Nx],
  with in[ci, z, ...] = 0 outside 0 <= z < Nz (circular in x and y, the
  periodic axes of a film; zero across the thickness);
* ReLU after every layer but the last; the network maps one channel (Q) to
  one channel (U) through ``width`` channels;
* the loss: mean over the counted voxels of (y - t)^2, and its gradient by
  back-propagation (the transposed layers and the weight correlations),
  written out as plain loops over the 27 offsets.

Arrays are [C, Z, Y, X].
"""
from __future__ import annotations

import numpy as np

OFFSETS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def shifted(a, dz, dy, dx):
    """s[..., z, y, x] = a[..., z + dz, (y + dy) mod Ny, (x + dx) mod Nx], zero
    where z + dz falls outside."""
    s = np.roll(a, shift=(-dy, -dx), axis=(-2, -1))
    out = np.zeros_like(s)
    nz = a.shape[-3]
    if dz >= 0:
        out[..., : nz - dz, :, :] = s[..., dz:, :, :]
    else:
        out[..., -dz:, :, :] = s[..., : nz + dz, :, :]
    return out


def layer(inp, W, b):
    """One 3x3x3 layer: inp [Ci, Z, Y, X], W [Co, Ci, 3, 3, 3], b [Co]."""
    co = W.shape[0]
    out = np.zeros((co,) + inp.shape[1:])
    for (dz, dy, dx) in OFFSETS:
        s = shifted(inp, dz, dy, dx)                     # [Ci, Z, Y, X]
        w = W[:, :, dz + 1, dy + 1, dx + 1]              # [Co, Ci]
        out += np.tensordot(w, s, axes=([1], [0]))
    return out + b[:, None, None, None]


def forward(x, params):
    """x [1, Z, Y, X] -> (y [1, Z, Y, X], activations for the backward pass).
    params: list of (W, b); ReLU after every layer but the last."""
    acts = [x]
    h = x
    for i, (W, b) in enumerate(params):
        z = layer(h, W, b)
        h = np.maximum(z, 0.0) if i + 1 < len(params) else z
        acts.append(h)
    return h, acts


def loss_and_grads(x, t, params, mask=None):
    """Mean squared error over the voxels where mask is true (all if None),
    and its gradient with respect to every W and b, by back-propagation:
    the gradient of a layer's input is the transposed layer (offsets
    reversed, channels swapped) applied to the gradient of its output, and
    the weight gradient correlates that output gradient with the shifted
    input."""
    y, acts = forward(x, params)
    m = np.ones(y.shape[1:], dtype=bool) if mask is None else mask
    cnt = float(m.sum())
    d = (y - t) * m
    loss = float(np.sum(d * d) / cnt)
    g = 2.0 * d / cnt                                    # dL/dy
    grads = [None] * len(params)
    for i in range(len(params) - 1, -1, -1):
        W, b = params[i]
        inp = acts[i]
        if i + 1 < len(params):
            g = g * (acts[i + 1] > 0)                    # through the ReLU
        gW = np.zeros_like(W)
        for (dz, dy, dx) in OFFSETS:
            s = shifted(inp, dz, dy, dx)
            gW[:, :, dz + 1, dy + 1, dx + 1] = np.tensordot(g, s, axes=([1, 2, 3], [1, 2, 3]))
        gb = g.sum(axis=(1, 2, 3))
        grads[i] = (gW, gb)
        # input gradient: in[ci, v] feeds out[co, v - o] through W[co, ci, o]
        gi = np.zeros_like(inp)
        for (dz, dy, dx) in OFFSETS:
            w = W[:, :, dz + 1, dy + 1, dx + 1]           # [Co, Ci]
            gi += shifted(np.tensordot(w, g, axes=([0], [0])), -dz, -dy, -dx)
        g = gi
    return loss, grads
