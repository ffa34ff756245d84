"""FP64 reference of the learned warm-start network pieces -- TEST INFRASTRUCTURE.

The warm start is an extension of the method: the paper itself starts its runs
from a Poisson solution or from an interpolated exact one (Sec. 2); here a small
3D convolution network predicts the potential instead.  Everything below is a
plain definition written out in NumPy, in FP64:

* conv3d: 3x3x3 correlation with zero padding ("same" size), channels last:
  out[b, z, y, x, co] = sum_{dz,dy,dx,ci} w[t, co, ci] * a[b, z+dz, y+dy, x+dx, ci],
  t = (dz+1)*9 + (dy+1)*3 + (dx+1), plus bias[co];
* its two backward products (input and weight gradients), checked by central
  finite differences in tests/test_oracle_nn.py;
* tanh and its derivative 1 - tanh^2;
* 2x2x2 mean restriction and cell-centred trilinear prolongation (weights 3/4
  and 1/4 per axis; at a face the missing coarse neighbour is extrapolated
  linearly, giving 5/4 and -1/4);
* Adam (Kingma & Ba) with bias correction;
* a training loss that adds to the mean-squared error the squared 7-point
  Laplacian (zero outside, index units) of one channel's error, and its
  gradient -- the residual of the predicted potential is what sets the
  solver's steps from a warm start, and it weighs fine-scale error heavily;
* the network's input features (density and coarse potential scaled by the
  sample's peak density, and the coarse potential's 7-point residual of the
  discrete Poisson equation, Eq. 1, with the second difference along an axis
  taken as 0 at the first and last cell) and the composition of the output
  into (phi, dphi/dt);
* bfloat16 round-to-nearest-even (for feeding the oracle the same rounded
  values as the device).
"""
from __future__ import annotations

import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def _shift(a: np.ndarray, dz: int, dy: int, dx: int) -> np.ndarray:
    """s[b, z, y, x, c] = a[b, z+dz, y+dy, x+dx, c], zero outside."""
    out = np.zeros_like(a)
    B, Z, Y, X, C = a.shape

    def rng(d, n):
        return (max(0, -d), min(n, n - d))

    z0, z1 = rng(dz, Z)
    y0, y1 = rng(dy, Y)
    x0, x1 = rng(dx, X)
    out[:, z0:z1, y0:y1, x0:x1, :] = a[:, z0 + dz:z1 + dz, y0 + dy:y1 + dy, x0 + dx:x1 + dx, :]
    return out


def conv3d(a: np.ndarray, w: np.ndarray, bias: np.ndarray | None = None) -> np.ndarray:
    """a: (B, Z, Y, X, Cin); w: (27, Cout, Cin); bias: (Cout,)."""
    B, Z, Y, X, Cin = a.shape
    Cout = w.shape[1]
    out = np.zeros((B, Z, Y, X, Cout))
    for t, (dz, dy, dx) in enumerate(TAPS):
        out += _shift(a, dz, dy, dx) @ w[t].T
    if bias is not None:
        out += bias
    return out


def conv3d_grad_input(g: np.ndarray, w: np.ndarray) -> np.ndarray:
    """d loss / d a given g = d loss / d out: sum_t shift(g, -tap) @ w[t]."""
    out = np.zeros(g.shape[:-1] + (w.shape[2],))
    for t, (dz, dy, dx) in enumerate(TAPS):
        out += _shift(g, -dz, -dy, -dx) @ w[t]
    return out


def conv3d_grad_weight(a: np.ndarray, g: np.ndarray) -> np.ndarray:
    """d loss / d w[t, co, ci] = sum_v g[v, co] a[v + tap, ci]."""
    Cin, Cout = a.shape[-1], g.shape[-1]
    dw = np.zeros((27, Cout, Cin))
    gf = g.reshape(-1, Cout)
    for t, (dz, dy, dx) in enumerate(TAPS):
        dw[t] = gf.T @ _shift(a, dz, dy, dx).reshape(-1, Cin)
    return dw


def conv3d_grad_bias(g: np.ndarray) -> np.ndarray:
    return g.reshape(-1, g.shape[-1]).sum(axis=0)


def tanh(x):
    return np.tanh(x)


def tanh_grad(y, g):
    """g * d tanh / d x expressed with y = tanh(x)."""
    return g * (1.0 - y * y)


def restrict2(f: np.ndarray) -> np.ndarray:
    """2x2x2 mean over the last three axes (..., Z, Y, X) -> (..., Z/2, Y/2, X/2)."""
    s = f.shape
    g = f.reshape(s[:-3] + (s[-3] // 2, 2, s[-2] // 2, 2, s[-1] // 2, 2))
    return g.mean(axis=(-5, -3, -1))


def _prolong_axis(c: np.ndarray, axis: int) -> np.ndarray:
    c = np.moveaxis(c, axis, -1)
    n = c.shape[-1]
    lo = np.empty_like(c)
    hi = np.empty_like(c)
    # fine cell 2i sits a quarter coarse cell left of coarse centre i, 2i+1 a quarter right
    left = np.concatenate([2 * c[..., :1] - c[..., 1:2] if n > 1 else c[..., :1], c[..., :-1]], axis=-1)
    right = np.concatenate([c[..., 1:], 2 * c[..., -1:] - c[..., -2:-1] if n > 1 else c[..., -1:]], axis=-1)
    lo[...] = 0.75 * c + 0.25 * left
    hi[...] = 0.75 * c + 0.25 * right
    f = np.stack([lo, hi], axis=-1).reshape(c.shape[:-1] + (2 * n,))
    return np.moveaxis(f, -1, axis)


def prolong2(c: np.ndarray) -> np.ndarray:
    """Cell-centred trilinear prolongation over the last three axes."""
    f = c
    for ax in (-3, -2, -1):
        f = _prolong_axis(f, ax)
    return f


def adam(p, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t starts at 1); returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def lap7(e: np.ndarray) -> np.ndarray:
    """7-point Laplacian in index units over the last three axes, zero outside:
    sum of the six neighbours minus 6 times the centre."""
    p = np.pad(e, [(0, 0)] * (e.ndim - 3) + [(1, 1)] * 3)
    c = p[..., 1:-1, 1:-1, 1:-1]
    return (p[..., :-2, 1:-1, 1:-1] + p[..., 2:, 1:-1, 1:-1] + p[..., 1:-1, :-2, 1:-1]
            + p[..., 1:-1, 2:, 1:-1] + p[..., 1:-1, 1:-1, :-2] + p[..., 1:-1, 1:-1, 2:] - 6.0 * c)


def lap_mse(out: np.ndarray, target: np.ndarray, ch: int, w: float):
    """out, target: (B, C, Z, Y, X).  loss = (sum e^2 + w sum (lap7 e_ch)^2) / e.size
    with e = out - target; returns (loss, d loss / d out)."""
    e = out - target
    r = lap7(e[:, ch])
    n = e.size
    loss = (np.sum(e * e) + w * np.sum(r * r)) / n
    g = 2.0 * e / n
    g[:, ch] += 2.0 * w * lap7(r) / n  # lap7 is symmetric (zero padding)
    return loss, g


def lap7_ext(f: np.ndarray) -> np.ndarray:
    """7-point Laplacian in index units over the last three axes; along each
    axis the second difference f[i-1] - 2 f[i] + f[i+1] is taken as 0 at the
    first and last cell (a linear extension across the faces)."""
    f = np.asarray(f, dtype=np.float64)
    out = np.zeros_like(f)
    for ax in (-3, -2, -1):
        n = f.shape[ax]
        if n < 3:
            continue
        fm = np.take(f, np.arange(0, n - 2), axis=ax)
        fc = np.take(f, np.arange(1, n - 1), axis=ax)
        fp = np.take(f, np.arange(2, n), axis=ax)
        d = fm - 2.0 * fc + fp
        idx = [slice(None)] * f.ndim
        idx[ax] = slice(1, n - 1)
        out[tuple(idx)] += d
    return out


def features(rho: np.ndarray, phi: np.ndarray, scale: np.ndarray, c: float) -> np.ndarray:
    """Inputs (B, 3, Z, Y, X) of the warm-start network from rho and a coarse
    potential phi (B, Z, Y, X) on a grid of spacing h, c = 4 pi G h^2, and the
    per-sample scale s (B,): rho / s, phi / s, (lap7_ext(phi) - c rho) / (c s)."""
    s = np.asarray(scale, dtype=np.float64).reshape(-1, 1, 1, 1)
    rho = np.asarray(rho, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    return np.stack([rho / s, phi / s, (lap7_ext(phi) - c * rho) / (c * s)], axis=1)


def compose(phi_c: np.ndarray, out: np.ndarray, scale: np.ndarray, out_scale: float):
    """(phi, dphi/dt) from the coarse potential (B, Z, Y, X) and the network
    output (B, 2, Z, Y, X) in units of s / out_scale."""
    f = np.asarray(scale, dtype=np.float64).reshape(-1, 1, 1, 1) / out_scale
    return phi_c + out[:, 0] * f, out[:, 1] * f


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round FP32 values to bfloat16 (nearest, ties to even); returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(x, layers):
    """Network: hidden layers tanh(conv + b), last layer linear.  Returns the
    list of activations [x, a1, ..., aL]."""
    acts = [x]
    for i, (w, b) in enumerate(layers):
        z = conv3d(acts[-1], w, b)
        acts.append(z if i == len(layers) - 1 else tanh(z))
    return acts


def backward(acts, layers, g_out):
    """Gradients of all (w, b) given d loss / d output."""
    grads = [None] * len(layers)
    g = g_out
    for i in range(len(layers) - 1, -1, -1):
        if i != len(layers) - 1:
            g = tanh_grad(acts[i + 1], g)
        grads[i] = (conv3d_grad_weight(acts[i], g), conv3d_grad_bias(g))
        if i > 0:
            g = conv3d_grad_input(g, layers[i][0])
    return grads
