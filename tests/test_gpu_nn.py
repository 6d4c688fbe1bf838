"""Warm-start network kernels against the FP64 reference (oracle/nnref.py),
called through the C ABI: each layer forward and backward on ragged shapes
with channel offsets, the whole U-Net's output and parameter gradients,
Adam, and a short training run that must lower the loss.

Tolerances follow from the arithmetic: inputs and weights are BF16 values
on both sides, products of two BF16 values are exact in FP32, so a layer
output differs from the FP64 value by its FP32 summation error (at most
n u32 sum|terms| for n terms, u32 = 2^-24) plus one rounding to BF16 (at
most 2^-8 relative).  Across the whole network, where the reference also
rounds every stored value to BF16, the two sides differ only where an FP32
summation error flips a BF16 rounding: a relative L2 difference of ~1e-3
is expected, 1e-2 (output) and 3e-2 (gradients) is asserted."""
import ctypes

import numpy as np
import pytest

from gpu_util import need_gpu, say
from oracle import nnref

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
BF = 2.0 ** -8


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _bits(a):
    """FP64 array of BF16-representable values -> int16 bit patterns."""
    a32 = np.ascontiguousarray(a, dtype=np.float32)
    return (a32.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)


def _vals(bits):
    return (bits.astype(np.int16).view(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _dev(a, dtype=None):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _host(t):
    return t.cpu().numpy()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _L():
    from paper_1405_2232_amd import nn
    return nn.lib()


def _embed(a, cs, co, rng):
    """Place channels of a (B, H, W, C) into a wider buffer at offset co,
    surrounded by unrelated BF16 values."""
    B, H, W, C = a.shape
    buf = nnref.bf16_round(rng.standard_normal((B, H, W, cs)))
    buf[..., co:co + C] = a
    return buf


SHAPES = [  # B, H, W, cin, cout, wrap, (xcs, xco), (ycs, yco)
    (2, 5, 70, 32, 48, 1, (40, 8), (52, 4)),
    (1, 9, 33, 16, 16, 0, (16, 0), (20, 4)),
    (3, 4, 64, 64, 128, 1, (64, 0), (128, 0)),
    (1, 6, 40, 32, 32, 0, (36, 4), (32, 0)),  # depth 32 but unaligned: the depth-16 path
]


@pytest.mark.parametrize("case", SHAPES, ids=lambda c: "%dx%dx%d_%d_%d_w%d" % c[:6])
def test_conv_forward_relu_and_input_gradient(case):
    import torch
    B, H, W, ci, co, wrap, (xcs, xco), (ycs, yco) = case
    rng = np.random.default_rng(11)
    x = nnref.bf16_round(rng.standard_normal((B, H, W, ci)))
    w = nnref.bf16_round(rng.standard_normal((co, 9, ci)) / np.sqrt(9 * ci))
    b = rng.standard_normal(co).astype(np.float32).astype(np.float64)
    xb = _dev(_bits(_embed(x, xcs, xco, rng)))
    wb = _dev(_bits(w))
    bb = _dev(b.astype(np.float32))
    yb = _dev(_bits(np.zeros((B, H, W, ycs))))
    say("case conv", case)
    for relu in (0, 1):
        rc = _L().lbmnn_conv3x3(_ptr(xb), xcs, xco, None, 0, 0, _ptr(wb), _ptr(bb), _ptr(yb), ycs, yco,
                                B, H, W, ci, co, relu, wrap, _stream())
        assert rc == 0
        torch.cuda.synchronize()
        got = _vals(_host(yb))[..., yco:yco + co]
        ref = nnref.conv3x3(x, w, b, wrap)
        mag = nnref.conv3x3(np.abs(x), np.abs(w), np.abs(b), wrap)
        if relu:
            ref = np.maximum(ref, 0)
        bound = BF * np.abs(ref) + (9 * ci + 1) * U32 * mag * (1 + BF) + 1e-30
        assert np.all(np.abs(got - ref) <= bound), float(np.max(np.abs(got - ref) / bound))
    # the input gradient: flipped weights through the same kernel, ReLU mask
    dy = nnref.bf16_round(rng.standard_normal((B, H, W, co)))
    mask = _vals(_host(yb))[..., yco:yco + co]  # a ReLU output (as a mask only)
    wt = _dev(_bits(np.zeros(9 * ci * co)))
    assert _L().lbmnn_conv3x3_flip(_ptr(wb), _ptr(wt), ci, co, _stream()) == 0
    dyb = _dev(_bits(_embed(dy, ycs, yco, rng)))
    mb = _dev(_bits(_embed(mask, ycs, yco, rng)))
    dxb = _dev(_bits(np.zeros((B, H, W, xcs))))
    rc = _L().lbmnn_conv3x3(_ptr(dyb), ycs, yco, _ptr(mb), ycs, yco, _ptr(wt), None, _ptr(dxb), xcs, xco,
                            B, H, W, co, ci, 0, wrap, _stream())
    assert rc == 0
    torch.cuda.synchronize()
    got = _vals(_host(dxb))[..., xco:xco + ci]
    dym = dy * (mask > 0)
    ref = nnref.conv3x3_back_input(dym, w, wrap)
    mag = nnref.conv3x3_back_input(np.abs(dym), np.abs(w), wrap)
    bound = BF * np.abs(ref) + 9 * co * U32 * mag * (1 + BF) + 1e-30
    assert np.all(np.abs(got - ref) <= bound), float(np.max(np.abs(got - ref) / bound))


@pytest.mark.parametrize("case", SHAPES, ids=lambda c: "%dx%dx%d_%d_%d_w%d" % c[:6])
def test_conv_weight_gradient(case):
    import torch
    B, H, W, ci, co, wrap, (xcs, xco), (ycs, yco) = case
    rng = np.random.default_rng(12)
    x = nnref.bf16_round(rng.standard_normal((B, H, W, ci)))
    dy = nnref.bf16_round(rng.standard_normal((B, H, W, co)))
    mask = nnref.bf16_round(rng.standard_normal((B, H, W, co)))
    xb = _dev(_bits(_embed(x, xcs, xco, rng)))
    dyb = _dev(_bits(_embed(dy, ycs, yco, rng)))
    mb = _dev(_bits(_embed(mask, ycs, yco, rng)))
    n = _L().lbmnn_wgrad_partials(B, H, W, ci, co)
    part = torch.empty(n, dtype=torch.float32, device="cuda")
    dw = torch.empty(co * 9 * ci, dtype=torch.float32, device="cuda")
    db = torch.empty(co, dtype=torch.float32, device="cuda")
    say("case wgrad", case)
    for use_mask in (False, True):
        rc = _L().lbmnn_conv3x3_wgrad(_ptr(xb), xcs, xco, _ptr(dyb), ycs, yco, _ptr(mb) if use_mask else None,
                                      ycs, yco, _ptr(dw), _ptr(db), _ptr(part), B, H, W, ci, co, wrap, _stream())
        assert rc == 0
        torch.cuda.synchronize()
        dym = dy * (mask > 0) if use_mask else dy
        rw, rb = nnref.conv3x3_back_weight(x, dym, wrap)
        mw, mbias = nnref.conv3x3_back_weight(np.abs(x), np.abs(dym), wrap)
        npix = B * H * W
        gw = _host(dw).reshape(co, 9, ci).astype(np.float64)
        gb = _host(db).astype(np.float64)
        assert np.all(np.abs(gw - rw) <= npix * U32 * mw + 1e-30)
        assert np.all(np.abs(gb - rb) <= npix * U32 * mbias + 1e-30)


def test_pool_upsample_and_their_backward():
    import torch
    rng = np.random.default_rng(13)
    B, H, W, C = 2, 6, 10, 12
    x = nnref.bf16_round(rng.standard_normal((B, H, W, C)))
    xb = _dev(_bits(_embed(x, 16, 4, rng)))
    yb = _dev(_bits(np.zeros((B, H // 2, W // 2, 20))))
    S = _stream()
    assert _L().lbmnn_pool2(_ptr(xb), 16, 4, _ptr(yb), 20, 8, B, H, W, C, S) == 0
    torch.cuda.synchronize()
    ref = nnref.pool2(x)
    got = _vals(_host(yb))[..., 8:8 + C]
    assert np.all(np.abs(got - ref) <= BF * np.abs(ref) + 4 * U32 * nnref.pool2(np.abs(x)))
    # backward accumulates into the existing gradient
    g0 = nnref.bf16_round(rng.standard_normal((B, H, W, C)))
    dy = nnref.bf16_round(rng.standard_normal((B, H // 2, W // 2, C)))
    gb = _dev(_bits(_embed(g0, 16, 4, rng)))
    dyb = _dev(_bits(_embed(dy, 20, 8, rng)))
    assert _L().lbmnn_pool2_back(_ptr(dyb), 20, 8, _ptr(gb), 16, 4, B, H, W, C, S) == 0
    torch.cuda.synchronize()
    ref = g0 + nnref.pool2_back(dy)
    got = _vals(_host(gb))[..., 4:4 + C]
    assert np.all(np.abs(got - ref) <= BF * np.abs(ref) + U32 * (np.abs(g0) + nnref.pool2_back(np.abs(dy))))
    # nearest upsampling and its backward (sum of four)
    ub = _dev(_bits(np.zeros((B, 2 * H, 2 * W, 16))))
    assert _L().lbmnn_up2(_ptr(xb), 16, 4, _ptr(ub), 16, 0, B, H, W, C, S) == 0
    torch.cuda.synchronize()
    assert np.array_equal(_vals(_host(ub))[..., :C], nnref.up2(x))
    d2 = nnref.bf16_round(rng.standard_normal((B, 2 * H, 2 * W, C)))
    d2b = _dev(_bits(_embed(d2, 16, 0, rng)))
    outb = _dev(_bits(np.zeros((B, H, W, C))))
    assert _L().lbmnn_up2_back(_ptr(d2b), 16, 0, _ptr(outb), C, 0, B, H, W, C, S) == 0
    torch.cuda.synchronize()
    ref = nnref.up2_back(d2)
    assert np.all(np.abs(_vals(_host(outb)) - ref) <= BF * np.abs(ref) + 4 * U32 * nnref.up2_back(np.abs(d2)))


def _net_case(seed, B=2, H=32, W=48):
    from paper_1405_2232_amd import inputs
    rng = np.random.default_rng(seed)
    Tc = inputs.cs_tc()
    rho = 0.15 + 0.1 * rng.standard_normal((B, H, W))
    T = Tc * (0.88 + 0.05 * rng.standard_normal((B, H, W)))
    s = np.column_stack([rng.uniform(0.85, 0.92, B), rng.uniform(0.7, 1.2, B), rng.uniform(0.6, 1.2, B)])
    tr = np.stack([0.3 * rng.standard_normal((B, H, W)), 0.3 * rng.standard_normal((B, H, W))], axis=-1)
    params = {}
    for name, shape in nnref.layer_shapes():
        if len(shape) == 3:
            params[name] = rng.standard_normal(shape) * np.sqrt(2.0 / (9 * shape[2]))
        else:
            params[name] = 0.1 * rng.standard_normal(shape)
    params = {k: v.astype(np.float32).astype(np.float64) for k, v in params.items()}
    return rho, T, s, tr, params, Tc


def test_unet_forward_and_gradients_match_reference():
    import torch
    from paper_1405_2232_amd import nn
    rho, T, s, target, params, Tc = _net_case(21)
    B, H, W = rho.shape
    net = nn.UNet(B, H, W, wrap_x=True, params=params)
    net.pack_input(_dev(rho), _dev(T), _dev(s), Tc)
    tgt = _dev(target.astype(np.float32))
    pred = _host(net.forward()).astype(np.float64)
    net.backward(tgt)
    loss = float(_host(net.loss_dev)[0])
    grads = net.get_grads()
    torch.cuda.synchronize()
    x0, base = nnref.pack_input(rho, T, s, Tc, nn.NORM_SHIFT, nn.NORM_SCALE)
    base = base.astype(np.float32).astype(np.float64)
    ref = nnref.Net(params, wrap_x=True, bf16=True)
    rpred = ref.forward(x0, base)
    rl = ref.loss(rpred, target.astype(np.float32).astype(np.float64))
    rg = ref.backward(rpred, target.astype(np.float32).astype(np.float64))
    e = np.linalg.norm(pred - rpred) / np.linalg.norm(rpred - base)
    say("unet output rel L2 (of the correction)", e, "loss", loss, rl)
    assert e < 1e-2
    assert abs(loss - rl) <= 1e-2 * rl
    worst = 0.0
    for name, _ in nnref.layer_shapes():
        d = np.linalg.norm(grads[name] - rg[name]) / (np.linalg.norm(rg[name]) + 1e-30)
        worst = max(worst, d)
        assert d < 3e-2, (name, d)
    say("unet worst gradient rel L2", worst)


def test_adam_matches_reference():
    import torch
    rng = np.random.default_rng(31)
    n = 1000
    w = rng.standard_normal(n).astype(np.float32)
    wd = _dev(w)
    w16 = torch.empty(n, dtype=torch.int16, device="cuda")
    m = torch.zeros(n, dtype=torch.float32, device="cuda")
    v = torch.zeros(n, dtype=torch.float32, device="cuda")
    rw, rm, rv = w.astype(np.float64), np.zeros(n), np.zeros(n)
    for t in range(1, 6):
        g = rng.standard_normal(n).astype(np.float32)
        assert _L().lbmnn_adam(_ptr(wd), _ptr(w16), _ptr(_dev(g)), _ptr(m), _ptr(v), n, 1e-2, 0.9, 0.999, 1e-8,
                               t, _stream()) == 0
        rw, rm, rv = nnref.adam_step(rw, g.astype(np.float64), rm, rv, t, 1e-2)
    torch.cuda.synchronize()
    got = _host(wd).astype(np.float64)
    assert np.max(np.abs(got - rw)) < 1e-5
    assert np.array_equal(_host(w16), _bits(nnref.bf16_round(got)))


def test_training_lowers_the_loss():
    import torch
    from paper_1405_2232_amd import nn
    rho, T, s, target, _, Tc = _net_case(41, B=4, H=32, W=32)
    net = nn.UNet(4, 32, 32)
    net.pack_input(_dev(rho), _dev(T), _dev(s), Tc)
    tgt = _dev(target.astype(np.float32))
    losses = []
    for it in range(60):
        net.forward()
        net.backward(tgt)
        losses.append(float(_host(net.loss_dev)[0]))
        net.adam(3e-3)
    torch.cuda.synchronize()
    say("training loss", losses[0], losses[-1])
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.5 * losses[0]
