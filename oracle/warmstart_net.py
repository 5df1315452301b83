"""FP64 reference of the network of the learned Poisson warm start (test infrastructure:
only tests use it).

A stack of 3 x 3 x 3 convolutions over a lattice [z][y][x] (periodic in x and y; in z
periodic, or zero beyond the first and last plane), channels ch[0] -> ch[1] -> ... -> 1, bias
on every layer and ReLU on all but the last.  Parameters are laid out per layer as the
weights [cout][cin][27] (tap k = (dz + 1) 9 + (dy + 1) 3 + (dx + 1)) followed by the bias
[cout].  The loss is the mean square difference to a target; its gradient is taken by
central finite differences in FP64, which is what the library's back-propagation is checked
against.
"""
from __future__ import annotations

import numpy as np

TAPS = [(k // 9 - 1, (k // 3) % 3 - 1, k % 3 - 1) for k in range(27)]


def shifted(a, dz, dy, dx, zwalls):
    """s[..., z, y, x] = a[..., z + dz, y + dy, x + dx], periodic in x and y; in z periodic or
    zero outside."""
    s = np.roll(a, (-dy, -dx), axis=(-2, -1))
    if not zwalls:
        return np.roll(s, -dz, axis=-3)
    out = np.zeros_like(s)
    nz = a.shape[-3]
    if dz == 0:
        out[...] = s
    elif dz > 0:
        out[..., : nz - dz, :, :] = s[..., dz:, :, :]
    else:
        out[..., -dz:, :, :] = s[..., : nz + dz, :, :]
    return out


def layers(params, ch):
    out, o = [], 0
    for l in range(len(ch) - 1):
        cin, cout = ch[l], ch[l + 1]
        w = np.asarray(params[o:o + cout * cin * 27], dtype=np.float64).reshape(cout, cin, 27)
        o += cout * cin * 27
        b = np.asarray(params[o:o + cout], dtype=np.float64)
        o += cout
        out.append((w, b))
    assert o == len(params)
    return out


def forward(params, ch, x, zwalls):
    """x: [cin][nz][ny][nx] -> [1][nz][ny][nx]."""
    a = np.asarray(x, dtype=np.float64)
    L = layers(params, ch)
    for l, (w, b) in enumerate(L):
        y = np.zeros((w.shape[0],) + a.shape[1:])
        for k, (dz, dy, dx) in enumerate(TAPS):
            y += np.einsum("oc,c...->o...", w[:, :, k], shifted(a, dz, dy, dx, zwalls))
        y += b[:, None, None, None]
        a = np.maximum(y, 0.0) if l + 1 < len(L) else y
    return a


def loss(params, ch, x, t, zwalls):
    d = forward(params, ch, x, zwalls) - np.asarray(t, dtype=np.float64)
    return float(np.mean(d * d))


def fd_gradient(params, ch, x, t, zwalls, indices, h=1e-6):
    """Central differences of the loss with respect to the chosen parameters."""
    p = np.asarray(params, dtype=np.float64).copy()
    g = []
    for i in indices:
        v = p[i]
        p[i] = v + h
        lp = loss(p, ch, x, t, zwalls)
        p[i] = v - h
        lm = loss(p, ch, x, t, zwalls)
        p[i] = v
        g.append((lp - lm) / (2 * h))
    return np.array(g)
