"""Plain FP64 reference of the warm-start network (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU baseline use this
module; the library's network runs on its own GPU kernels and never calls
it.  Everything here is NumPy in FP64, written from the textbook
definitions of the layers (no passage of the paper defines them):

- 3x3 convolution, "same" size, zero boundary in y, periodic or zero in x:
  y(p, o) = b(o) + sum_{tap, i} w(o, tap, i) x(p + off(tap), i),
  off(tap) = (tap // 3 - 1, tap % 3 - 1) in (y, x);
- ReLU; 2x2 average pooling; nearest 2x upsampling; channel concatenation;
- output layer pred = base + bh + wh f (1x1, C -> 2) and the mean squared
  error over both output channels;
- the backward pass of each layer, written as the adjoint (scatter) of its
  forward map, and Adam with bias correction.

`bf16=True` rounds every stored activation, activation gradient and conv
weight to BF16 (round to nearest even) at the same places the GPU stores
them, so that both sides take their rounding decisions on nearly the same
values; with `bf16=False` the network is exact FP64 (used for the finite-
difference gradient pins).
"""
import numpy as np


def bf16_round(a):
    """Round to the nearest BF16 value (ties to even), returned as FP64."""
    a32 = np.ascontiguousarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    finite = (u & 0x7F800000) != 0x7F800000
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    r = np.where(finite, r, u & 0xFFFF0000)
    return r.astype(np.uint32).view(np.float32).astype(np.float64).reshape(np.shape(a))


def _pad(x, wrap_x):
    """(B, H, W, C) -> (B, H+2, W+2, C): zeros in y, wrap or zeros in x."""
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    if wrap_x:
        xp[:, 1:-1, 0] = x[:, :, -1]
        xp[:, 1:-1, -1] = x[:, :, 0]
    return xp


def conv3x3(x, w, b=None, wrap_x=True):
    """x (B, H, W, Cin), w (Cout, 9, Cin) -> (B, H, W, Cout)."""
    B, H, W, _ = x.shape
    xp = _pad(x, wrap_x)
    out = np.zeros((B, H, W, w.shape[0]))
    for tap in range(9):
        ky, kx = divmod(tap, 3)
        out += xp[:, ky:ky + H, kx:kx + W, :] @ w[:, tap, :].T
    if b is not None:
        out += b
    return out


def conv3x3_back_input(dy, w, wrap_x=True):
    """Adjoint of conv3x3 in x: scatter dy (B, H, W, Cout) back through
    every tap."""
    B, H, W, _ = dy.shape
    dxp = np.zeros((B, H + 2, W + 2, w.shape[2]))
    for tap in range(9):
        ky, kx = divmod(tap, 3)
        dxp[:, ky:ky + H, kx:kx + W, :] += dy @ w[:, tap, :]
    if wrap_x:
        dxp[:, 1:-1, 1] += dxp[:, 1:-1, -1]
        dxp[:, 1:-1, -2] += dxp[:, 1:-1, 0]
    return dxp[:, 1:-1, 1:-1, :]


def conv3x3_back_weight(x, dy, wrap_x=True):
    """dw (Cout, 9, Cin) and db (Cout,) of conv3x3 given its input x and dy."""
    B, H, W, _ = x.shape
    xp = _pad(x, wrap_x)
    dw = np.zeros((dy.shape[3], 9, x.shape[3]))
    for tap in range(9):
        ky, kx = divmod(tap, 3)
        sl = xp[:, ky:ky + H, kx:kx + W, :]
        dw[:, tap, :] = np.einsum("bhwo,bhwi->oi", dy, sl)
    return dw, dy.sum(axis=(0, 1, 2))


def pool2(x):
    B, H, W, C = x.shape
    return x.reshape(B, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def pool2_back(dy):
    return np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2) * 0.25


def up2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up2_back(dy):
    B, H, W, C = dy.shape
    return dy.reshape(B, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


# network: encoder levels (conv, conv) with 2x2 pooling between them, a
# bottleneck, decoder levels (upsample, concatenate the encoder output of
# the same level after the upsampled channels, conv, conv), 1x1 output
# layer added to the first two input channels
ENC = [(16, 32), (32, 32), (32, 64)]
MID = 64
DEC = [(64 + 64, 64), (64 + 32, 32), (32 + 32, 32)]  # deepest level first


def layer_shapes():
    """Ordered (name, shape) of every parameter."""
    out = []
    for lvl, (ci, co) in enumerate(ENC):
        out += [("enc%d_a.w" % lvl, (co, 9, ci)), ("enc%d_a.b" % lvl, (co,)),
                ("enc%d_b.w" % lvl, (co, 9, co)), ("enc%d_b.b" % lvl, (co,))]
    ci = ENC[-1][1]
    out += [("mid_a.w", (MID, 9, ci)), ("mid_a.b", (MID,)),
            ("mid_b.w", (MID, 9, MID)), ("mid_b.b", (MID,))]
    for k, (ci, co) in enumerate(DEC):
        lvl = len(DEC) - 1 - k
        out += [("dec%d_a.w" % lvl, (co, 9, ci)), ("dec%d_a.b" % lvl, (co,)),
                ("dec%d_b.w" % lvl, (co, 9, co)), ("dec%d_b.b" % lvl, (co,))]
    out += [("head.w", (2, DEC[-1][1])), ("head.b", (2,))]
    return out


def pack_input(rho, T, scalars, tc, shift, scale):
    """Input planes (B, H, W, 16) and base (B, H, W, 2) from FP64 fields
    rho, T (B, H, W) and per-image scalars (B, 3) = (T0/T_c, tau_f, tau_g)."""
    B, H, W = rho.shape
    x = np.zeros((B, H, W, 16))
    x[..., 0] = (rho - shift[0]) / scale[0]
    x[..., 1] = (T / tc - shift[1]) / scale[1]
    for k in range(3):
        x[..., 2 + k] = ((scalars[:, k] - shift[2 + k]) / scale[2 + k])[:, None, None]
    return x, x[..., :2].copy()


def pack_target(rho, T, tc, shift, scale):
    return np.stack([(rho - shift[0]) / scale[0], (T / tc - shift[1]) / scale[1]], axis=-1)


class Net:
    """FP64 forward/backward of the network for parameters `params`
    (dict name -> array, shapes from layer_shapes())."""

    def __init__(self, params, wrap_x=True, bf16=False):
        self.p = {k: np.asarray(v, dtype=np.float64) for k, v in params.items()}
        self.wrap_x = wrap_x
        self.bf16 = bf16
        self.r = bf16_round if bf16 else (lambda a: a)
        # conv weights are stored in BF16; biases and the output layer in FP32
        self.w = {k: (self.r(v) if (k.endswith(".w") and not k.startswith("head")) else v)
                  for k, v in self.p.items()}

    def _conv(self, name, x):
        y = conv3x3(x, self.w[name + ".w"], self.w[name + ".b"], self.wrap_x)
        return self.r(np.maximum(y, 0.0))

    def forward(self, x0, base):
        r = self.r
        c = {"x0": r(x0)}
        h = c["x0"]
        skips = []
        for lvl in range(len(ENC)):
            c["enc%d_a" % lvl] = a = self._conv("enc%d_a" % lvl, h)
            c["enc%d_b" % lvl] = s = self._conv("enc%d_b" % lvl, a)
            skips.append(s)
            h = r(pool2(s))
            c["pool%d" % lvl] = h
        c["mid_a"] = a = self._conv("mid_a", h)
        c["mid_b"] = h = self._conv("mid_b", a)
        for lvl in reversed(range(len(ENC))):
            cat = np.concatenate([up2(h), skips[lvl]], axis=-1)
            c["cat%d" % lvl] = cat
            c["dec%d_a" % lvl] = a = self._conv("dec%d_a" % lvl, cat)
            c["dec%d_b" % lvl] = h = self._conv("dec%d_b" % lvl, a)
        pred = base + self.p["head.b"] + h @ self.p["head.w"].T
        self.cache = c
        return pred

    def loss(self, pred, target):
        return float(np.mean((pred - target) ** 2))

    def backward(self, pred, target):
        """Gradients of the mean squared error wrt every parameter."""
        r, c, g = self.r, self.cache, {}
        f = c["dec0_b"]
        dpred = 2.0 * (pred - target) / pred.size
        g["head.w"] = np.einsum("bhwc,bhwk->ck", dpred, f)
        g["head.b"] = dpred.sum(axis=(0, 1, 2))
        dh = r(dpred @ self.p["head.w"])

        def conv_back(name, x, y, dy, need_dx=True):
            dyp = dy * (y > 0)
            g[name + ".w"], g[name + ".b"] = conv3x3_back_weight(x, dyp, self.wrap_x)
            return r(conv3x3_back_input(dyp, self.w[name + ".w"], self.wrap_x)) if need_dx else None

        dskip = {}
        for lvl in range(len(ENC)):
            da = conv_back("dec%d_b" % lvl, c["dec%d_a" % lvl], c["dec%d_b" % lvl], dh)
            dcat = conv_back("dec%d_a" % lvl, c["cat%d" % lvl], c["dec%d_a" % lvl], da)
            nup = dcat.shape[-1] - c["enc%d_b" % lvl].shape[-1]
            dskip[lvl] = dcat[..., nup:]
            dh = r(up2_back(dcat[..., :nup]))
        da = conv_back("mid_b", c["mid_a"], c["mid_b"], dh)
        dh = conv_back("mid_a", c["pool%d" % (len(ENC) - 1)], c["mid_a"], da)
        for lvl in reversed(range(len(ENC))):
            ds = r(dskip[lvl] + pool2_back(dh))
            da = conv_back("enc%d_b" % lvl, c["enc%d_a" % lvl], c["enc%d_b" % lvl], ds)
            x_in = c["pool%d" % (lvl - 1)] if lvl > 0 else c["x0"]
            dh = conv_back("enc%d_a" % lvl, x_in, c["enc%d_a" % lvl], da, need_dx=lvl > 0)
        return g


def adam_step(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (bias-corrected); returns new (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
