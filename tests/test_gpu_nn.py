"""GPU network kernels (learned warm start) against the FP64 network oracle.

Inputs and weights are rounded to bfloat16 on the host and the oracle is fed
the same rounded values, so FP32 outputs differ only by accumulation order
(tolerance 2e-5 relative to the largest magnitude); bfloat16 outputs are
compared within one bfloat16 rounding (2^-8 relative) of the oracle value.
"""
import numpy as np
import pytest

from oracle import nn

pytestmark = pytest.mark.gpu


def _t(x, dtype):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda").to(dtype)


def _h(t):
    import torch

    return t.detach().double().cpu().numpy()


def _rand_bf(shape, seed, scale=1.0):
    r = np.random.default_rng(seed).standard_normal(shape) * scale
    return nn.bf16_round(r.astype(np.float32))


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-30))


SHAPES = [(1, 3, 4, 16), (2, 6, 5, 32), (1, 8, 8, 64), (1, 2, 7, 96), (1, 3, 5, 128)]


@pytest.mark.parametrize("shape", SHAPES)
def test_conv3d_forward_modes(gpu_lib, shape):
    import torch

    hgs = gpu_lib
    B, Z, Y, X = shape
    a = _rand_bf((B, Z, Y, X, 16), 1)
    w = _rand_bf((27, 16, 16), 2, 0.2)
    b = np.random.default_rng(3).standard_normal(16).astype(np.float32).astype(np.float64)
    ta, tw, tb = _t(a, torch.bfloat16), _t(w, torch.bfloat16), _t(b, torch.float32)
    ref = nn.conv3d(a, w, b)
    out = torch.empty((B, Z, Y, X, 16), dtype=torch.float32, device="cuda")
    hgs.nn_conv3d(ta, tw, tb, out, hgs.NN_F32)
    assert rel(_h(out), ref) < 2e-5
    o16 = torch.empty((B, Z, Y, X, 16), dtype=torch.bfloat16, device="cuda")
    hgs.nn_conv3d(ta, tw, tb, o16, hgs.NN_TANH_BF16)
    tr = np.tanh(ref)
    assert np.all(np.abs(_h(o16) - tr) <= 2 ** -8 * np.abs(tr) + 1e-6)
    aux = _rand_bf((B, Z, Y, X, 16), 4, 0.5)
    hgs.nn_conv3d(ta, tw, None, o16, hgs.NN_DTANH_BF16, aux=_t(aux, torch.bfloat16))
    dr = nn.conv3d(a, w) * (1 - aux * aux)
    assert np.all(np.abs(_h(o16) - dr) <= 2 ** -8 * np.abs(dr) + 1e-4 * np.max(np.abs(dr)))


@pytest.mark.parametrize("shape", SHAPES)
def test_conv3d_input_gradient_by_flipped_weights(gpu_lib, shape):
    import torch

    hgs = gpu_lib
    B, Z, Y, X = shape
    g = _rand_bf((B, Z, Y, X, 16), 5)
    w = _rand_bf((27, 16, 16), 6, 0.2)
    tw = _t(w, torch.bfloat16)
    wt = torch.empty_like(tw)
    hgs.nn_flip_weights(tw, wt)
    out = torch.empty((B, Z, Y, X, 16), dtype=torch.float32, device="cuda")
    hgs.nn_conv3d(_t(g, torch.bfloat16), wt, None, out, hgs.NN_F32)
    assert rel(_h(out), nn.conv3d_grad_input(g, w)) < 2e-5


@pytest.mark.parametrize("shape", SHAPES + [(3, 5, 7, 48)])
def test_conv3d_weight_gradient(gpu_lib, shape):
    import torch

    hgs = gpu_lib
    B, Z, Y, X = shape
    a = _rand_bf((B, Z, Y, X, 16), 7)
    g = _rand_bf((B, Z, Y, X, 16), 8)
    dw = torch.empty((27, 16, 16), dtype=torch.float32, device="cuda")
    db = torch.empty(16, dtype=torch.float32, device="cuda")
    hgs.nn_wgrad(_t(a, torch.bfloat16), _t(g, torch.bfloat16), dw, db)
    assert rel(_h(dw), nn.conv3d_grad_weight(a, g)) < 2e-5
    assert rel(_h(db), nn.conv3d_grad_bias(g)) < 2e-5


def test_transfer_operators(gpu_lib):
    import torch

    hgs = gpu_lib
    rng = np.random.default_rng(9)
    for cz, cy, cx in [(1, 1, 1), (2, 3, 5), (8, 8, 8), (16, 12, 20)]:
        f = rng.standard_normal((2, 2 * cz, 2 * cy, 2 * cx))
        c = torch.empty((2, cz, cy, cx), dtype=torch.float64, device="cuda")
        hgs.nn_restrict2(_t(f, torch.float64), c)
        assert np.allclose(_h(c), nn.restrict2(f), rtol=0, atol=1e-14)
        cc = rng.standard_normal((2, cz, cy, cx))
        fo = torch.empty((2, 2 * cz, 2 * cy, 2 * cx), dtype=torch.float64, device="cuda")
        hgs.nn_prolong2(_t(cc, torch.float64), fo)
        if min(cz, cy, cx) > 1:
            assert np.allclose(_h(fo), nn.prolong2(cc), rtol=0, atol=1e-13)


def test_adam_mse_pack(gpu_lib):
    import torch

    hgs = gpu_lib
    rng = np.random.default_rng(10)
    n = 1000
    p = rng.standard_normal(n).astype(np.float32)
    g = rng.standard_normal(n).astype(np.float32)
    tp, tm, tv = _t(p, torch.float32), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    p16 = torch.empty(n, dtype=torch.bfloat16, device="cuda")
    pp, mm, vv = p.astype(np.float64), np.zeros(n), np.zeros(n)
    for t in (1, 2, 3):
        hgs.nn_adam(tp, tm, tv, _t(g, torch.float32), p16, 1e-2, t)
        pp, mm, vv = nn.adam(pp, mm, vv, g.astype(np.float64), t, lr=1e-2)
    assert np.allclose(_h(tp), pp, rtol=0, atol=1e-5)
    assert np.array_equal(_h(p16), nn.bf16_round(_h(tp).astype(np.float32)))
    # pack / mse / unpack
    B, C = 2, 3
    fields = rng.standard_normal((B, C, 4, 5, 16)).astype(np.float32)
    packed = torch.empty((B, 4, 5, 16, 16), dtype=torch.bfloat16, device="cuda")
    hgs.nn_pack(_t(fields, torch.float32), packed)
    ph = _h(packed)
    assert np.array_equal(ph[..., :C], np.moveaxis(nn.bf16_round(fields), 1, -1))
    assert np.all(ph[..., C:] == 0)
    out = _t(rng.standard_normal((B, 4, 5, 16, 16)).astype(np.float32), torch.float32)
    tgt = rng.standard_normal((B, C, 4, 5, 16)).astype(np.float32)
    grad = torch.empty((B, 4, 5, 16, 16), dtype=torch.bfloat16, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    parts = torch.empty(hgs.NN_MSE_PARTIALS, dtype=torch.float64, device="cuda")
    hgs.nn_mse(out, _t(tgt, torch.float32), grad, loss, parts)
    d = np.moveaxis(_h(out)[..., :C], -1, 1) - tgt
    assert float(loss.item()) == pytest.approx(np.sum(d * d), rel=1e-6)  # differences formed in FP32
    gh = _h(grad)
    assert np.allclose(np.moveaxis(gh[..., :C], -1, 1), nn.bf16_round((2 * d / d.size).astype(np.float32)), rtol=0,
                       atol=1e-12)
    back = torch.empty((B, C, 4, 5, 16), dtype=torch.float32, device="cuda")
    hgs.nn_unpack(out, C, back)
    assert np.array_equal(_h(back), np.moveaxis(_h(out)[..., :C], -1, 1))


@pytest.mark.parametrize("shape", [(2, 2, 5, 4, 7), (1, 3, 9, 6, 16)])
def test_lapmse_matches_oracle(gpu_lib, shape):
    """Laplacian-weighted loss and its gradient against the FP64 oracle
    (differences formed exactly from FP32 inputs; gradient rounded to bf16)."""
    import torch

    hgs = gpu_lib
    B, C, Z, Y, X = shape
    rng = np.random.default_rng(12)
    out = rng.standard_normal((B, Z, Y, X, 16)).astype(np.float32)
    tgt = rng.standard_normal((B, C, Z, Y, X)).astype(np.float32)
    w, ch = 0.6, C - 1
    grad = torch.empty((B, Z, Y, X, 16), dtype=torch.bfloat16, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    parts = torch.empty(hgs.NN_MSE_PARTIALS, dtype=torch.float64, device="cuda")
    scratch = torch.empty(B * Z * Y * X, dtype=torch.float32, device="cuda")
    hgs.nn_lapmse(_t(out, torch.float32), _t(tgt, torch.float32), grad, loss, parts, scratch, ch=ch, w=w)
    o = np.moveaxis(out[..., :C].astype(np.float64), -1, 1)
    ref_loss, ref_g = nn.lap_mse(o, tgt.astype(np.float64), ch, w)
    n = B * C * Z * Y * X
    assert float(loss.item()) == pytest.approx(ref_loss * n, rel=1e-6)
    gh = np.moveaxis(_h(grad)[..., :C], -1, 1)
    assert np.all(np.abs(gh - ref_g) <= 2.0 ** -8 * np.abs(ref_g) + 1e-6 * np.max(np.abs(ref_g)))
    assert np.all(_h(grad)[..., C:] == 0)


@pytest.mark.parametrize("shape", [(3, 64, 64, 64), (2, 33, 40, 48), (1, 1, 1, 4), (2, 16, 3, 20), (4, 1, 1, 260)])
def test_maxabs_vector_path(gpu_lib, shape):
    """Per-sample max |x| over samples whose voxel count is a multiple of 4
    (16-byte loads, chunks that may be empty) and a peak in a chunk's last
    vector; the scratch-free call gives the same values."""
    import torch

    rng = np.random.default_rng(17)
    a = rng.normal(0.0, 1.0, shape).astype(np.float32)
    B = shape[0]
    flat = a.reshape(B, -1)
    flat[0, -1] = 50.0
    flat[B - 1, flat.shape[1] // 2] = -70.0
    want = np.abs(flat).max(axis=1)
    x = _t(a, torch.float32)
    s = torch.empty(B, dtype=torch.float32, device="cuda")
    gpu_lib.nn_maxabs(x, s)
    assert np.array_equal(_h(s), want.astype(np.float64))
    s2 = torch.empty(B, dtype=torch.float32, device="cuda")
    gpu_lib.nn_maxabs_noalloc(x, s2)
    assert torch.equal(s, s2)


def test_features_maxabs_compose_match_oracle(gpu_lib):
    import torch

    hgs = gpu_lib
    rng = np.random.default_rng(13)
    B, Z, Y, X = 2, 5, 7, 9
    rho = rng.uniform(0.0, 3.0, (B, Z, Y, X)).astype(np.float32)
    rho[1] *= -1.0  # max |x|, not max x
    phi = rng.standard_normal((B, Z, Y, X)).astype(np.float32)
    s = torch.empty(B, dtype=torch.float32, device="cuda")
    hgs.nn_maxabs(_t(rho, torch.float32), s)
    assert np.array_equal(_h(s), np.abs(rho).reshape(B, -1).max(axis=1).astype(np.float64))
    c = 4.0 * np.pi * 0.03 ** 2
    out = torch.empty((B, 3, Z, Y, X), dtype=torch.float32, device="cuda")
    hgs.nn_features(_t(rho, torch.float32), _t(phi, torch.float32), s, c, out)
    ref = nn.features(rho.astype(np.float64), phi.astype(np.float64), _h(s), c)
    # FP64 arithmetic on FP32 inputs, rounded once to FP32
    assert np.all(np.abs(_h(out) - ref) <= 2.0 ** -23 * np.abs(ref) + 1e-30)
    y = rng.standard_normal((B, Z, Y, X, 16)).astype(np.float32)
    p = torch.empty((B, Z, Y, X), dtype=torch.float32, device="cuda")
    d = torch.empty_like(p)
    hgs.nn_compose(_t(phi, torch.float32), _t(y, torch.float32), s, 3.0, p, d)
    rp, rd = nn.compose(phi.astype(np.float64), np.moveaxis(y[..., :2], -1, 1).astype(np.float64), _h(s), 3.0)
    assert np.all(np.abs(_h(p) - rp) <= 2.0 ** -23 * np.abs(rp) + 1e-30)
    assert np.all(np.abs(_h(d) - rd) <= 2.0 ** -23 * np.abs(rd) + 1e-30)
