"""Pins of the FP64 warm-start network reference (oracle/net.py) against
independent definitions: scipy's 2-D cross-correlation, central finite
differences of the loss, closed forms of Adam's first step, adjointness,
exact bilinear cases and exact bfloat16 rounding cases."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import net


def rng(seed=0):
    return np.random.default_rng(seed)


@pytest.mark.parametrize("stride", [1, 2])
def test_conv_matches_scipy_correlate(stride):
    r = rng(1)
    x = r.standard_normal((2, 8, 10, 3))
    w = r.standard_normal((4, 3, 3, 3))
    b = r.standard_normal(4)
    z = net.conv3x3(x, w, b, stride)
    assert z.shape == (2, 8 // stride, 10 // stride, 4)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(correlate2d(x[n, :, :, c], w[o, :, :, c], mode="same")
                             for c in range(3))
            np.testing.assert_allclose(z[n, :, :, o], ref[::stride, ::stride], rtol=0, atol=1e-12)


def test_conv_single_tap_brute_force():
    # one non-zero weight at tap (ky, kx) = (0, 2) shifts the input by (-1, +1)
    x = np.arange(2 * 6 * 6 * 1, dtype=float).reshape(2, 6, 6, 1)
    w = np.zeros((1, 3, 3, 1))
    w[0, 0, 2, 0] = 2.0
    z = net.conv3x3(x, w, np.zeros(1), 1)
    for n in range(2):
        for i in range(6):
            for j in range(6):
                src = (i - 1, j + 1)
                exp = 2.0 * x[n, src[0], src[1], 0] if 0 <= src[0] < 6 and 0 <= src[1] < 6 else 0.0
                assert z[n, i, j, 0] == exp


def test_silu_and_grad():
    z = np.linspace(-6, 6, 101)
    np.testing.assert_allclose(net.silu(z), z * 0.5 * (1 + np.tanh(z / 2)), atol=1e-15)
    h = 1e-6
    fd = (net.silu(z + h) - net.silu(z - h)) / (2 * h)
    np.testing.assert_allclose(net.silu_grad(z), fd, atol=1e-9)


def test_upsample_adjoint():
    r = rng(2)
    x = r.standard_normal((2, 3, 4, 5))
    y = r.standard_normal((2, 6, 8, 5))
    assert abs(np.vdot(net.upsample2(x), y) - np.vdot(x, net.upsample2_backward(y))) < 1e-12
    assert np.array_equal(net.upsample2(x)[:, 5, 7], x[:, 2, 3])


TINY = dict(widths=(3, 4, 5, 6, 7), cin=2, cout=3, res=16)


def tiny_net(seed=3):
    r = rng(seed)
    npar = net.param_count(TINY["widths"], TINY["cin"], TINY["cout"])
    flat = r.standard_normal(npar) * 0.4
    x = r.standard_normal((2, TINY["res"], TINY["res"], TINY["cin"]))
    t = r.standard_normal((2, TINY["res"], TINY["res"], 3))
    return flat, x, t


def loss_of(flat, x, t):
    y, _ = net.forward(flat, x, TINY["widths"], TINY["cout"])
    return net.mse(y, t)[0]


def test_param_layout():
    assert net.param_count((32, 32, 64, 64, 128), 8, 8) == 281088 + 520  # weights + biases
    flat = np.arange(net.param_count((3, 4, 5, 6, 7), 2, 3), dtype=float)
    P = net.unflatten(flat, (3, 4, 5, 6, 7), 2, 3)
    assert P[0][0].shape == (3, 3, 3, 2) and P[0][1][0] == 54 and P[1][0][0, 0, 0, 0] == 57
    assert P[5][0].shape == (6, 3, 3, 7) and P[9][0].shape == (3, 3, 3, 3)


def test_backward_matches_central_differences():
    flat, x, t = tiny_net()
    y, cache = net.forward(flat, x, TINY["widths"], TINY["cout"])
    _, dy = net.mse(y, t)
    g = net.backward(flat, cache, dy, TINY["widths"], TINY["cout"])
    h = 1e-6
    fd = np.empty_like(flat)
    for k in range(flat.size):
        p, m = flat.copy(), flat.copy()
        p[k] += h
        m[k] -= h
        fd[k] = (loss_of(p, x, t) - loss_of(m, x, t)) / (2 * h)
    err = np.abs(fd - g).max() / np.abs(g).max()
    assert err <= 1e-6, err
    # every layer's weights and biases receive a non-trivial gradient
    k = 0
    for o, i, _, _ in net.layer_shapes(TINY["widths"], TINY["cin"], TINY["cout"]):
        assert np.abs(g[k:k + o * 9 * i]).max() > 0 and np.abs(g[k + o * 9 * i:k + o * 9 * i + o]).max() > 0
        k += o * 9 * i + o


def test_stride2_geometry_against_stride1():
    # the stride-2 conv equals the stride-1 conv sampled at even pixels; its
    # input gradient equals the stride-1 input gradient of the zero-filled dz
    r = rng(4)
    x = r.standard_normal((1, 8, 8, 2))
    w = r.standard_normal((3, 3, 3, 2))
    dz2 = r.standard_normal((1, 4, 4, 3))
    dz1 = np.zeros((1, 8, 8, 3))
    dz1[:, ::2, ::2] = dz2
    a = net.conv3x3_backward(x, w, dz2, 2)
    b = net.conv3x3_backward(x, w, dz1, 1)
    for u, v in zip(a, b):
        np.testing.assert_allclose(u, v, atol=1e-12)


def test_adam_first_step_closed_form():
    r = rng(5)
    w0 = r.standard_normal(50)
    g = r.standard_normal(50)
    w1, m, v = net.adam_step(w0, np.zeros(50), np.zeros(50), g, 1, lr=1e-3)
    # bias-corrected moments of the first step are g and g^2: each weight moves
    # by lr against the sign of its gradient (up to eps)
    np.testing.assert_allclose(w1 - w0, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    # scale invariance of the update (eps aside)
    w1s, _, _ = net.adam_step(w0, np.zeros(50), np.zeros(50), 1000 * g, 1, lr=1e-3)
    np.testing.assert_allclose(w1s, w1, atol=1e-10)
    # a constant gradient keeps the step at lr (up to eps) for every t
    w, m, v = w0.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 6):
        wn, m, v = net.adam_step(w, m, v, g, t, lr=1e-3)
        np.testing.assert_allclose(wn - w, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-9)
        w = wn


def test_bilinear_exact_cases():
    r = rng(6)
    src = r.standard_normal((12, 20))
    np.testing.assert_array_equal(net.bilinear(src, 12, 20), src)
    # halving each dimension averages 2 x 2 blocks of cell centres
    half = net.bilinear(src, 6, 10)
    np.testing.assert_allclose(half, src.reshape(6, 2, 10, 2).mean(axis=(1, 3)), atol=1e-14)
    # an affine function of the cell-centre coordinates is reproduced wherever
    # the destination centre lies inside the source centres
    sy, sx = (np.arange(12) + 0.5) / 12, (np.arange(20) + 0.5) / 20
    f = 0.3 + 1.7 * sx[None, :] - 0.9 * sy[:, None]
    d = net.bilinear(f, 31, 47)
    dy, dx = (np.arange(31) + 0.5) / 31, (np.arange(47) + 0.5) / 47
    ex = 0.3 + 1.7 * np.clip(dx, sx[0], sx[-1])[None, :] - 0.9 * np.clip(dy, sy[0], sy[-1])[:, None]
    np.testing.assert_allclose(d, ex, atol=1e-13)


def test_bf16_rounding_cases():
    e = 2.0 ** -8
    vals = np.array([1.0, 1 + e, 1 + 3 * e, 1 + 1.5 * e, -2.0 - 2 * 2 * e * 0.5, 3.0e38])
    exp = np.array([1.0, 1.0, 1 + 4 * e, 1 + 2 * e, -2.0, 2.9975e38])
    got = net.bf16_round(vals)
    np.testing.assert_array_equal(got[:5], exp[:5])
    assert abs(got[5] - 3.0e38) / 3.0e38 < 2 ** -8


def test_net_inputs_channels():
    x = net.net_inputs([[6.0, 7.0, 4.0], [3.0, 0.71, 1.0]], 4)
    assert x.shape == (2, 4, 4, 8)
    np.testing.assert_allclose(x[0, 2, :, 0], [0.125, 0.375, 0.625, 0.875])
    np.testing.assert_allclose(x[0, :, 1, 1], [0.125, 0.375, 0.625, 0.875])
    np.testing.assert_allclose(x[:, 0, 0, 2:5], [[1.0, 1.0, 1.0], [-1.0, -1.0, 0.25]])
    assert np.all(x[..., 5:] == 0)
