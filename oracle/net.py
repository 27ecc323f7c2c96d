"""Plain FP64 numpy reference of the warm-start network and its data path.

TEST INFRASTRUCTURE ONLY (same rule as the rest of ``oracle/``): it checks
the GPU library and is never called by it.  Everything here is written from
the textbook definitions, one operation per function, with no fusion:

* conv3x3: 3 x 3 cross-correlation, zero padding 1, stride 1 or 2
  (output pixel (oy, ox) is centred on input pixel (s*oy, s*ox));
* SiLU activation z * sigmoid(z);
* nearest-neighbour x2 upsampling;
* mean squared error over the three target channels;
* Adam (Kingma and Ba, 2015) with bias correction;
* bilinear resampling between cell-centred grids on the unit square.

Not part of the paper: the network is the learned initial guess for the
steady-state solver.  Layouts: activations NHWC, weights [Cout][3][3][Cin].

Network (encoder-decoder with additive skips), widths w0..w4:
  e0 = silu(conv(x, s1))          R      w0
  e1 = silu(conv(e0, s2))         R/2    w1
  e2 = silu(conv(e1, s2))         R/4    w2
  e3 = silu(conv(e2, s2))         R/8    w3
  e4 = silu(conv(e3, s2))         R/16   w4
  d3 = silu(conv(up(e4))) + e3    R/8    w3
  d2 = silu(conv(up(d3))) + e2    R/4    w2
  d1 = silu(conv(up(d2))) + e1    R/2    w1
  d0 = silu(conv(up(d1))) + e0    R      w0
  y  = conv(d0)                   R      cout (linear)
"""
from __future__ import annotations

import numpy as np

# ---------------------------------------------------------------- layers


def conv3x3(x, w, b, stride):
    """z[n, oy, ox, o] = b[o] + sum_{ky, kx, c} xpad[n, s*oy + ky, s*ox + kx, c] w[o, ky, kx, c]."""
    n, h, wd, c = x.shape
    ho, wo = h // stride, wd // stride
    xp = np.zeros((n, h + 2, wd + 2, c))
    xp[:, 1:-1, 1:-1, :] = x
    z = np.zeros((n, ho, wo, w.shape[0])) + b
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + stride * ho:stride, kx:kx + stride * wo:stride, :]
            z += patch @ w[:, ky, kx, :].T
    return z


def conv3x3_backward(x, w, dz, stride):
    """Gradients of conv3x3 with respect to x, w and b, given dL/dz."""
    n, h, wd, c = x.shape
    ho, wo = h // stride, wd // stride
    xp = np.zeros((n, h + 2, wd + 2, c))
    xp[:, 1:-1, 1:-1, :] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + stride * ho:stride, kx:kx + stride * wo:stride, :]
            dw[:, ky, kx, :] = np.einsum("nhwo,nhwc->oc", dz, patch)
            dxp[:, ky:ky + stride * ho:stride, kx:kx + stride * wo:stride, :] += dz @ w[:, ky, kx, :]
    return dxp[:, 1:-1, 1:-1, :], dw, dz.sum(axis=(0, 1, 2))


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def upsample2(x):
    return x.repeat(2, axis=1).repeat(2, axis=2)


def upsample2_backward(dy):
    n, h, w, c = dy.shape
    return dy.reshape(n, h // 2, 2, w // 2, 2, c).sum(axis=(2, 4))


# ---------------------------------------------------------------- network


def layer_shapes(widths, cin, cout):
    """(Cout, Cin, stride, upsample-before) of the ten convolutions in order."""
    w0, w1, w2, w3, w4 = widths
    return [(w0, cin, 1, False), (w1, w0, 2, False), (w2, w1, 2, False), (w3, w2, 2, False),
            (w4, w3, 2, False),
            (w3, w4, 1, True), (w2, w3, 1, True), (w1, w2, 1, True), (w0, w1, 1, True),
            (cout, w0, 1, False)]


def param_count(widths, cin, cout):
    return sum(o * 9 * i + o for o, i, _, _ in layer_shapes(widths, cin, cout))


def unflatten(flat, widths, cin, cout):
    """Flat parameter vector -> list of (w [o,3,3,i], b [o]); per layer the
    weights come first, then the bias."""
    out, k = [], 0
    for o, i, _, _ in layer_shapes(widths, cin, cout):
        w = flat[k:k + o * 9 * i].reshape(o, 3, 3, i)
        k += o * 9 * i
        b = flat[k:k + o]
        k += o
        out.append((w, b))
    assert k == flat.size
    return out


def forward(flat, x, widths, cout):
    """Returns y and the cache the backward pass needs."""
    P = unflatten(np.asarray(flat, np.float64), widths, x.shape[3], cout)
    shapes = layer_shapes(widths, x.shape[3], cout)
    cache = {"x_in": [], "z": []}
    h = x
    enc = []
    for li in range(5):
        _, _, s, _ = shapes[li]
        cache["x_in"].append(h)
        z = conv3x3(h, *P[li], s)
        cache["z"].append(z)
        h = silu(z)
        enc.append(h)
    for li, skip in zip(range(5, 9), (3, 2, 1, 0)):
        u = upsample2(h)
        cache["x_in"].append(u)
        z = conv3x3(u, *P[li], 1)
        cache["z"].append(z)
        h = silu(z) + enc[skip]
    cache["x_in"].append(h)
    y = conv3x3(h, *P[9], 1)
    return y, cache


def mse(y, t, nch=3):
    """Mean over batch, pixels and the first nch channels of (y - t)^2, and
    dL/dy (zero on the padding channels)."""
    d = y[..., :nch] - t
    loss = float(np.mean(d * d))
    dy = np.zeros_like(y)
    dy[..., :nch] = 2.0 * d / d.size
    return loss, dy


def backward(flat, cache, dy, widths, cout):
    """Flat gradient vector of the loss for dL/dy, in the layout of ``flat``."""
    cin = cache["x_in"][0].shape[3]
    P = unflatten(np.asarray(flat, np.float64), widths, cin, cout)
    shapes = layer_shapes(widths, cin, cout)
    grads = [None] * 10
    dx, dw, db = conv3x3_backward(cache["x_in"][9], P[9][0], dy, 1)
    grads[9] = (dw, db)
    da = dx                      # dL/d d0
    skip_grad = {}
    for li, skip in zip(range(8, 4, -1), (0, 1, 2, 3)):
        skip_grad[skip] = da     # d_k = silu(z) + e_k
        dz = da * silu_grad(cache["z"][li])
        du, dw, db = conv3x3_backward(cache["x_in"][li], P[li][0], dz, 1)
        grads[li] = (dw, db)
        da = upsample2_backward(du)   # dL/d of the previous decoder level (or e4)
    for li in range(4, -1, -1):
        if li < 4:
            da = da + skip_grad[li]
        dz = da * silu_grad(cache["z"][li])
        dx, dw, db = conv3x3_backward(cache["x_in"][li], P[li][0], dz, shapes[li][2])
        grads[li] = (dw, db)
        da = dx
    return np.concatenate([np.concatenate([g[0].ravel(), g[1].ravel()]) for g in grads])


def adam_step(w, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns new (w, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return w - lr * mhat / (np.sqrt(vhat) + eps), m, v


# ---------------------------------------------------------------- data path


def net_inputs(feat, res, cin=8):
    """Input planes for samples feat[k] = (log10 Ra, Pr, aspect A): channels
    X, Y (cell centres on the unit square), (log10 Ra - 4.5) / 1.5,
    (Pr - 3.855) / 3.145, A / 4; padding channels zero.  NHWC."""
    feat = np.atleast_2d(np.asarray(feat, np.float64))
    c = (np.arange(res) + 0.5) / res
    x = np.zeros((feat.shape[0], res, res, cin))
    x[..., 0] = c[None, None, :]
    x[..., 1] = c[None, :, None]
    x[..., 2] = ((feat[:, 0] - 4.5) / 1.5)[:, None, None]
    x[..., 3] = ((feat[:, 1] - 3.855) / 3.145)[:, None, None]
    x[..., 4] = (feat[:, 2] / 4.0)[:, None, None]
    return x


def bilinear(src, dny, dnx):
    """Resample a cell-centred [sny][snx] field to [dny][dnx] on the same
    rectangle: the destination centre (i + 1/2)/dnx maps to the source index
    coordinate (i + 1/2) snx/dnx - 1/2, clamped to [0, snx - 1]; same in y."""
    sny, snx = src.shape

    def coords(dn, sn):
        q = np.clip((np.arange(dn) + 0.5) * sn / dn - 0.5, 0.0, sn - 1.0)
        i0 = np.minimum(np.floor(q).astype(int), sn - 1)
        i1 = np.minimum(i0 + 1, sn - 1)
        return i0, i1, q - i0

    y0, y1, fy = coords(dny, sny)
    x0, x1, fx = coords(dnx, snx)
    a = src[np.ix_(y0, x0)] * (1 - fx)[None, :] + src[np.ix_(y0, x1)] * fx[None, :]
    b = src[np.ix_(y1, x0)] * (1 - fx)[None, :] + src[np.ix_(y1, x1)] * fx[None, :]
    return a * (1 - fy)[:, None] + b * fy[:, None]


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(a, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
