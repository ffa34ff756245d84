"""Pins of the FP64 network oracle (no GPU): finite differences, a direct
correlation loop, closed forms for the transfer operators and Adam."""
import numpy as np
import pytest

from oracle import nn


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def test_conv_matches_direct_loop():
    a = _rand((1, 4, 5, 3, 2), 1)
    w = _rand((27, 3, 2), 2)
    b = _rand((3,), 3)
    out = nn.conv3d(a, w, b)
    B, Z, Y, X, C = a.shape
    ref = np.zeros((1, Z, Y, X, 3))
    for z in range(Z):
        for y in range(Y):
            for x in range(X):
                for co in range(3):
                    s = b[co]
                    for t, (dz, dy, dx) in enumerate(nn.TAPS):
                        zz, yy, xx = z + dz, y + dy, x + dx
                        if 0 <= zz < Z and 0 <= yy < Y and 0 <= xx < X:
                            s += np.dot(w[t, co], a[0, zz, yy, xx])
                    ref[0, z, y, x, co] = s
    assert np.allclose(out, ref, rtol=1e-13, atol=1e-13)


def test_conv_gradients_finite_differences():
    a = _rand((2, 3, 4, 5, 3), 4)
    w = _rand((27, 2, 3), 5)
    b = _rand((2,), 6)
    g = _rand((2, 3, 4, 5, 2), 7)
    loss = lambda a_, w_, b_: np.sum(nn.conv3d(a_, w_, b_) * g)
    ga = nn.conv3d_grad_input(g, w)
    gw = nn.conv3d_grad_weight(a, g)
    gb = nn.conv3d_grad_bias(g)
    h = 1e-6
    rng = np.random.default_rng(8)
    for _ in range(12):
        idx = tuple(rng.integers(0, s) for s in a.shape)
        d = np.zeros_like(a)
        d[idx] = h
        fd = (loss(a + d, w, b) - loss(a - d, w, b)) / (2 * h)
        assert fd == pytest.approx(ga[idx], rel=1e-7, abs=1e-7)
    for _ in range(12):
        idx = tuple(rng.integers(0, s) for s in w.shape)
        d = np.zeros_like(w)
        d[idx] = h
        fd = (loss(a, w + d, b) - loss(a, w - d, b)) / (2 * h)
        assert fd == pytest.approx(gw[idx], rel=1e-7, abs=1e-7)
    for co in range(2):
        d = np.zeros_like(b)
        d[co] = h
        fd = (loss(a, w, b + d) - loss(a, w, b - d)) / (2 * h)
        assert fd == pytest.approx(gb[co], rel=1e-7, abs=1e-7)


def test_network_backward_finite_differences():
    rng = np.random.default_rng(9)
    x = rng.standard_normal((1, 4, 4, 4, 2))
    layers = [(0.3 * rng.standard_normal((27, 3, 2)), 0.1 * rng.standard_normal(3)),
              (0.3 * rng.standard_normal((27, 3, 3)), 0.1 * rng.standard_normal(3)),
              (0.3 * rng.standard_normal((27, 2, 3)), 0.1 * rng.standard_normal(2))]
    tgt = rng.standard_normal((1, 4, 4, 4, 2))

    def loss(ls):
        out = nn.forward(x, ls)[-1]
        return 0.5 * np.sum((out - tgt) ** 2)

    acts = nn.forward(x, layers)
    grads = nn.backward(acts, layers, acts[-1] - tgt)
    h = 1e-6
    for li in range(3):
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in layers[li][0].shape)
            lp = [(w.copy(), b.copy()) for w, b in layers]
            lm = [(w.copy(), b.copy()) for w, b in layers]
            lp[li][0][idx] += h
            lm[li][0][idx] -= h
            fd = (loss(lp) - loss(lm)) / (2 * h)
            assert fd == pytest.approx(grads[li][0][idx], rel=1e-6, abs=1e-8)


def test_restrict_and_prolong_closed_forms():
    n = 8
    c = (np.arange(n) + 0.5) / n  # coarse cell centres on [0, 1]
    f = (np.arange(2 * n) + 0.5) / (2 * n)
    Zc, Yc, Xc = np.meshgrid(c, c, c, indexing="ij")
    Zf, Yf, Xf = np.meshgrid(f, f, f, indexing="ij")
    lin = lambda X, Y, Z: 1.5 * X - 0.7 * Y + 0.2 * Z + 0.3
    # prolongation is exact on linear fields (including the extrapolated faces)
    assert np.allclose(nn.prolong2(lin(Xc, Yc, Zc)), lin(Xf, Yf, Zf), rtol=0, atol=1e-13)
    # restriction of a linear field equals the field at coarse centres
    assert np.allclose(nn.restrict2(lin(Xf, Yf, Zf)), lin(Xc, Yc, Zc), rtol=0, atol=1e-13)
    # along one axis, restriction after prolongation is the stencil 3/4 c_i + 1/8 (c_{i-1} + c_{i+1})
    r = np.random.default_rng(3).standard_normal(9)
    field = np.broadcast_to(r, (2, 2, 9)).copy()
    rp = nn.restrict2(nn.prolong2(field))[0, 0]
    assert np.allclose(rp[1:-1], 0.75 * r[1:-1] + 0.125 * (r[:-2] + r[2:]), rtol=0, atol=1e-14)
    # interior weights 3/4, 1/4 along one axis
    e = np.zeros((3, 3, 3))
    e[1, 1, 1] = 1.0
    p = nn.prolong2(e)
    assert p[2, 2, 2] == pytest.approx(0.75 ** 3)
    assert p[1, 2, 2] == pytest.approx(0.25 * 0.75 ** 2)


def test_adam_matches_closed_form_first_step():
    p = np.array([1.0, -2.0])
    g = np.array([0.5, -3.0])
    p1, m, v = nn.adam(p, np.zeros(2), np.zeros(2), g, 1, lr=0.1)
    # at t = 1 the bias-corrected step is lr * sign(g) (up to eps)
    assert np.allclose(p1, p - 0.1 * np.sign(g), rtol=0, atol=1e-7)


def test_bf16_round():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 3.14159265], dtype=np.float32)
    r = nn.bf16_round(x)
    assert r[0] == 1.0
    assert r[1] == 1.0  # tie goes to even
    assert r[2] == 1.0 + 2 ** -6
    assert r[3] == -2.5
    assert abs(r[4] - 3.140625) < 1e-12


def test_lap7_and_lap_mse_gradient():
    # lap7 of a quadratic in the interior is its constant Laplacian (index units)
    z, y, x = np.meshgrid(np.arange(5.0), np.arange(6.0), np.arange(7.0), indexing="ij")
    q = (x ** 2 + 2 * y ** 2 - 0.5 * z ** 2)[None]
    assert np.allclose(nn.lap7(q)[0, 1:-1, 1:-1, 1:-1], 2 + 4 - 1, rtol=0, atol=1e-12)
    # at a corner the zero padding drops the three outside neighbours
    e = np.zeros((1, 3, 3, 3))
    e[0, 0, 0, 0] = 1.0
    assert nn.lap7(e)[0, 0, 0, 0] == -6.0 and nn.lap7(e)[0, 1, 0, 0] == 1.0
    # gradient by central differences
    rng = np.random.default_rng(11)
    out = rng.standard_normal((2, 2, 4, 3, 5))
    tgt = rng.standard_normal((2, 2, 4, 3, 5))
    loss, g = nn.lap_mse(out, tgt, 0, 0.7)
    h = 1e-6
    for _ in range(16):
        idx = tuple(rng.integers(0, s) for s in out.shape)
        d = np.zeros_like(out)
        d[idx] = h
        fd = (nn.lap_mse(out + d, tgt, 0, 0.7)[0] - nn.lap_mse(out - d, tgt, 0, 0.7)[0]) / (2 * h)
        assert fd == pytest.approx(g[idx], rel=1e-6, abs=1e-9)
    # w = 0 is the plain mean-squared error
    assert nn.lap_mse(out, tgt, 0, 0.0)[0] == pytest.approx(np.mean((out - tgt) ** 2), rel=1e-14)


def test_lap7_ext_and_features_pins():
    z, y, x = np.meshgrid(np.arange(6.0), np.arange(5.0), np.arange(7.0), indexing="ij")
    # linear fields: the linear extension across the faces makes it exact (0)
    lin = (0.3 * x - 1.2 * y + 2.0 * z + 0.7)[None]
    assert np.allclose(nn.lap7_ext(lin), 0.0, atol=1e-12)
    # x^2: 2 in the interior along x, 0 on the first and last cell of x
    q = (x ** 2)[None]
    L = nn.lap7_ext(q)[0]
    assert np.allclose(L[:, :, 1:-1], 2.0) and np.allclose(L[:, :, [0, -1]], 0.0)
    # the residual feature of the discrete Poisson solution vanishes at cells
    # whose 7-point stencil lies inside the grid (Eq. 1 in discrete form)
    from oracle import core, poisson
    g = core.Grid.cube(16)
    xc, yc, zc = (c[1:-1] for c in g.centres())
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    rho = np.exp(-((X - 0.1) ** 2 + Y ** 2 + (Z + 0.2) ** 2) / 0.05)
    P = core.padded(g)
    core.boundary(g, core.moments(g, rho, 4), 4, 1.0, P)
    phi = poisson.solve_dst(g, rho, 1.0, P)
    c = 4.0 * np.pi * g.dx ** 2
    f = nn.features(rho[None], phi[None], np.array([rho.max()]), c)
    assert f.shape == (1, 3, 16, 16, 16)
    assert np.allclose(f[0, 0], rho / rho.max()) and np.allclose(f[0, 1], phi / rho.max())
    assert np.max(np.abs(f[0, 2, 1:-1, 1:-1, 1:-1])) < 1e-10
    assert np.max(np.abs(f[0, 2])) > 1e-3  # the face cells see the truncated stencil
    # compose inverts the scaling
    out = np.random.default_rng(0).standard_normal((1, 2, 16, 16, 16))
    p, d = nn.compose(phi[None], out, np.array([2.0]), 4.0)
    assert np.allclose(p, phi[None] + 0.5 * out[:, 0]) and np.allclose(d, 0.5 * out[:, 1])
