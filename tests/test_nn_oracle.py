"""Pins of the FP64 network reference against definitions it does not
share code with: SciPy's 2-D correlation, adjoint identities of the linear
layers, central finite differences of the whole network's loss, the closed
form of a first Adam step and exactly representable BF16 roundings."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import nnref


def _rng(seed):
    return np.random.default_rng(seed)


def test_bf16_round_ties_to_even():
    one = 1.0
    ulp = 2.0 ** -7  # BF16 keeps 7 explicit mantissa bits
    vals = np.array([one, one + ulp / 2, one + 1.5 * ulp, one + 0.75 * ulp, -3.0 - ulp / 4, 0.0])
    want = np.array([one, one, one + 2 * ulp, one + ulp, -3.0, 0.0])
    assert np.array_equal(nnref.bf16_round(vals), want)


@pytest.mark.parametrize("wrap_x", [False, True])
def test_conv3x3_matches_scipy_correlation(wrap_x):
    rng = _rng(1)
    B, H, W, ci, co = 2, 7, 9, 3, 4
    x = rng.standard_normal((B, H, W, ci))
    w = rng.standard_normal((co, 9, ci))
    b = rng.standard_normal(co)
    got = nnref.conv3x3(x, w, b, wrap_x)
    want = np.zeros_like(got)
    for bb in range(B):
        for o in range(co):
            acc = np.full((H, W), b[o])
            for i in range(ci):
                img = x[bb, :, :, i]
                img = np.pad(img, ((1, 1), (0, 0)))
                img = np.pad(img, ((0, 0), (1, 1)), mode="wrap" if wrap_x else "constant")
                acc += correlate2d(img, w[o, :, i].reshape(3, 3), mode="valid")
            want[bb, :, :, o] = acc
    assert np.max(np.abs(got - want)) < 1e-12


@pytest.mark.parametrize("wrap_x", [False, True])
def test_conv_backward_is_the_adjoint(wrap_x):
    rng = _rng(2)
    B, H, W, ci, co = 2, 6, 8, 5, 3
    x = rng.standard_normal((B, H, W, ci))
    w = rng.standard_normal((co, 9, ci))
    y = rng.standard_normal((B, H, W, co))
    lhs = np.sum(nnref.conv3x3(x, w, None, wrap_x) * y)
    assert abs(lhs - np.sum(x * nnref.conv3x3_back_input(y, w, wrap_x))) < 1e-11 * (1 + abs(lhs))
    dw, db = nnref.conv3x3_back_weight(x, y, wrap_x)
    assert abs(lhs - np.sum(w * dw)) < 1e-11 * (1 + abs(lhs))
    assert np.allclose(db, y.sum(axis=(0, 1, 2)), rtol=0, atol=1e-12)


def test_pool_and_upsample_adjoints():
    rng = _rng(3)
    x = rng.standard_normal((2, 8, 6, 4))
    y = rng.standard_normal((2, 4, 3, 4))
    assert abs(np.sum(nnref.pool2(x) * y) - np.sum(x * nnref.pool2_back(y))) < 1e-12
    assert abs(np.sum(nnref.up2(y) * x) - np.sum(y * nnref.up2_back(x))) < 1e-12
    # averages and copies of constants
    assert np.allclose(nnref.pool2(np.full((1, 4, 4, 1), 3.0)), 3.0)
    assert np.array_equal(nnref.up2(y)[:, ::2, 1::2], y)


def _small_params(seed):
    rng = _rng(seed)
    p = {}
    for name, shape in nnref.layer_shapes():
        # activations of order one through the depth of the network
        scale = np.sqrt(2.0 / (9 * shape[2])) if len(shape) == 3 else 0.1
        p[name] = rng.standard_normal(shape) * scale
    return p


def test_network_gradient_matches_finite_differences():
    """Central differences of the exact FP64 loss against the backward pass
    for entries of every parameter tensor."""
    rng = _rng(4)
    B, H, W = 1, 16, 16
    x0 = rng.standard_normal((B, H, W, 16))
    x0[..., 5:] = 0.0
    base = x0[..., :2].copy()
    target = rng.standard_normal((B, H, W, 2))
    params = _small_params(5)
    net = nnref.Net(params, wrap_x=True)
    pred = net.forward(x0, base)
    g = net.backward(pred, target)
    h = 1e-5
    worst = 0.0
    for name, shape in nnref.layer_shapes():
        flat = np.prod(shape)
        for k in rng.choice(flat, size=min(3, flat), replace=False):
            idx = np.unravel_index(k, shape)
            vals = []
            for sgn in (1, -1):
                q = {kk: v.copy() for kk, v in params.items()}
                q[name][idx] += sgn * h
                n2 = nnref.Net(q, wrap_x=True)
                vals.append(n2.loss(n2.forward(x0, base), target))
            fd = (vals[0] - vals[1]) / (2 * h)
            # rounding of the differenced loss is ~1e-16 / h; truncation O(h^2)
            err = abs(fd - g[name][idx]) / (abs(fd) + abs(g[name][idx]) + 1e-6)
            worst = max(worst, err)
            assert err < 1e-5, (name, idx, fd, g[name][idx])
    assert worst < 1e-5


def test_untrained_zero_head_returns_input():
    rng = _rng(6)
    p = _small_params(7)
    p["head.w"][:] = 0.0
    p["head.b"][:] = 0.0
    x0 = rng.standard_normal((2, 8, 8, 16))
    base = x0[..., :2].copy()
    assert np.array_equal(nnref.Net(p).forward(x0, base), base)


def test_adam_first_step_closed_form():
    g = np.array([0.5, -2.0, 1e-3])
    w, m, v = nnref.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.1, eps=1e-8)
    assert np.allclose(w, -0.1 * g / (np.abs(g) + 1e-8), rtol=1e-14, atol=0)
    # constant gradient: the bias-corrected moments stay g and g^2
    for t in range(2, 5):
        w2, m, v = nnref.adam_step(w, g, m, v, t, lr=0.1, eps=1e-8)
        assert np.allclose(w2 - w, -0.1 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
        w = w2


def test_pack_input_normalisation():
    rho = np.full((1, 4, 4), 0.25)
    T = np.full((1, 4, 4), 0.09)
    s = np.array([[0.9, 1.0, 0.8]])
    x, base = nnref.pack_input(rho, T, s, 0.1, (0.15, 0.88, 0.88, 0.95, 0.9), (0.1, 0.05, 0.05, 0.25, 0.3))
    assert np.allclose(x[0, 0, 0, :5], [1.0, 0.4, 0.4, 0.2, -1.0 / 3.0])
    assert np.all(x[..., 5:] == 0) and np.array_equal(base, x[..., :2])
