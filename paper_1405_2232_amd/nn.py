"""Warm-start network on the GPU: binding of include/lbmnn.h (argument
marshalling) and the U-Net built from those kernels.

The network maps an initial state of a thermal two-phase run (density,
temperature, and the run's T0/T_c, tau_f, tau_g as constant planes) to a
near-steady density and temperature.  Every layer, its backward pass, the
loss and the optimizer run in the library's HIP kernels (BF16 activations
and weights, FP32 accumulation and optimizer state); PyTorch only holds
the buffers and supplies the stream.  There is no CPU fallback.
"""
import ctypes

import numpy as np

from .lbm import LbmError, lib as _lbm_lib

# input planes: rho, T/T_c, T0/T_c, tau_f, tau_g (value - shift) / scale
NORM_SHIFT = (0.15, 0.88, 0.88, 0.95, 0.9)
NORM_SCALE = (0.1, 0.05, 0.05, 0.25, 0.3)
IN_CH = 16  # five planes padded to a multiple of 16 with zeros

# encoder levels (cin, cout), bottleneck width, decoder levels deepest first
# (cin = upsampled + skip channels, cout)
ENC = [(16, 32), (32, 32), (32, 64)]
MID = 64
DEC = [(64 + 64, 64), (64 + 32, 32), (32 + 32, 32)]

_sig_done = False


def lib():
    global _sig_done
    L = _lbm_lib()
    if not _sig_done:
        vp, i, sz, f, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t, ctypes.c_float, ctypes.c_double
        fp = ctypes.POINTER(ctypes.c_float)
        sig = {
            "lbmnn_conv3x3": [vp, i, i, vp, i, i, vp, vp, vp, i, i, i, i, i, i, i, i, i, vp],
            "lbmnn_conv3x3_flip": [vp, vp, i, i, vp],
            "lbmnn_conv3x3_wgrad": [vp, i, i, vp, i, i, vp, i, i, vp, vp, vp, i, i, i, i, i, i, vp],
            "lbmnn_pool2": [vp, i, i, vp, i, i, i, i, i, i, vp],
            "lbmnn_pool2_back": [vp, i, i, vp, i, i, i, i, i, i, vp],
            "lbmnn_up2": [vp, i, i, vp, i, i, i, i, i, i, vp],
            "lbmnn_up2_back": [vp, i, i, vp, i, i, i, i, i, i, vp],
            "lbmnn_pack_input": [vp, vp, vp, d, fp, fp, vp, vp, i, i, i, vp],
            "lbmnn_pack_target": [vp, vp, d, fp, fp, vp, i, i, i, vp],
            "lbmnn_unpack_output": [vp, d, fp, fp, vp, vp, i, i, i, vp],
            "lbmnn_head": [vp, i, i, vp, vp, vp, vp, i, i, i, i, vp],
            "lbmnn_head_loss": [vp, i, i, vp, vp, vp, vp, vp, vp, vp, vp, i, i, vp, i, i, i, i, vp],
            "lbmnn_adam": [vp, vp, vp, vp, vp, sz, f, f, f, f, i, vp],
            "lbmnn_to_bf16": [vp, vp, sz, vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.lbmnn_wgrad_partials.argtypes = [i, i, i, i, i]
        L.lbmnn_wgrad_partials.restype = sz
        L.lbmnn_head_partials.argtypes = [i, i, i, i]
        L.lbmnn_head_partials.restype = sz
        _sig_done = True
    return L


def _chk(fn, rc):
    if rc != 0:
        raise LbmError(fn, rc)


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _floats(v):
    return (ctypes.c_float * len(v))(*v)


class Act:
    """A BF16 NHWC activation: buffer `buf` (int16 tensor [B, H, W, cs])
    and the channel window [co, co + C)."""

    def __init__(self, buf, co, C):
        self.buf, self.co, self.C = buf, co, C
        self.B, self.H, self.W, self.cs = buf.shape

    @property
    def ptr(self):
        return _p(self.buf)


def layer_shapes():
    out = []
    for lvl, (ci, co) in enumerate(ENC):
        out += [("enc%d_a.w" % lvl, (co, 9, ci)), ("enc%d_a.b" % lvl, (co,)),
                ("enc%d_b.w" % lvl, (co, 9, co)), ("enc%d_b.b" % lvl, (co,))]
    ci = ENC[-1][1]
    out += [("mid_a.w", (MID, 9, ci)), ("mid_a.b", (MID,)), ("mid_b.w", (MID, 9, MID)), ("mid_b.b", (MID,))]
    for k, (ci, co) in enumerate(DEC):
        lvl = len(DEC) - 1 - k
        out += [("dec%d_a.w" % lvl, (co, 9, ci)), ("dec%d_a.b" % lvl, (co,)),
                ("dec%d_b.w" % lvl, (co, 9, co)), ("dec%d_b.b" % lvl, (co,))]
    out += [("head.w", (2, DEC[-1][1])), ("head.b", (2,))]
    return out


def init_params(seed=0):
    """He-normal conv weights (fan-in of the real input channels), zero
    biases, zero output layer (the untrained network returns its input)."""
    rng = np.random.default_rng(seed)
    out = {}
    for name, shape in layer_shapes():
        if name.endswith(".b") or name.startswith("head"):
            out[name] = np.zeros(shape)
        else:
            fan_in = 9 * (5 if name.startswith("enc0_a") else shape[2])
            w = rng.standard_normal(shape) * np.sqrt(2.0 / fan_in)
            if name.startswith("enc0_a"):
                w[:, :, 5:] = 0.0
            out[name] = w
    return out


class UNet:
    """The network for batches of `B` images of H x W (H, W divisible by
    8), periodic in x when wrap_x.  Parameters live in one flat FP32
    buffer with a BF16 copy; gradients and Adam moments beside them."""

    def __init__(self, B, H, W, wrap_x=True, device="cuda", stream=None, params=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the warm-start network needs a ROCm GPU; none is visible")
        if H % 8 or W % 8:
            raise ValueError("H and W must be multiples of 8")
        self.B, self.H, self.W, self.wrap = B, H, W, int(bool(wrap_x))
        self.dev = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.dev)
        self.sp = ctypes.c_void_p(self.stream.cuda_stream)
        self.offs = {}
        n = 0
        for name, shape in layer_shapes():
            self.offs[name] = (n, shape)
            n += int(np.prod(shape))
            n = (n + 3) // 4 * 4
        self.nparam = n
        f32 = dict(dtype=torch.float32, device=self.dev)
        self.w32 = torch.zeros(n, **f32)
        self.w16 = torch.zeros(n, dtype=torch.int16, device=self.dev)
        self.g32 = torch.zeros(n, **f32)
        self.m = torch.zeros(n, **f32)
        self.v = torch.zeros(n, **f32)
        self.t = 0
        self._alloc()
        self.set_params(params if params is not None else init_params(0))

    # -- buffers ---------------------------------------------------------
    def _alloc(self):
        import torch
        B, H, W = self.B, self.H, self.W
        i16 = dict(dtype=torch.int16, device=self.dev)

        def act(lvl, C):
            return torch.empty((B, H >> lvl, W >> lvl, C), **i16)

        A = {}
        A["x0"] = act(0, IN_CH)
        cat_ch = [DEC[2][0], DEC[1][0], DEC[0][0]]  # per level 0, 1, 2
        for lvl, (ci, co) in enumerate(ENC):
            A["enc%d_a" % lvl] = act(lvl, co)
            A["cat%d" % lvl] = act(lvl, cat_ch[lvl])
            A["pool%d" % lvl] = act(lvl + 1, co)
        A["mid_a"] = act(3, MID)
        A["mid_b"] = act(3, MID)
        for k, (ci, co) in enumerate(DEC):
            lvl = len(DEC) - 1 - k
            A["dec%d_a" % lvl] = act(lvl, co)
            A["dec%d_b" % lvl] = act(lvl, co)
        self.A = A
        self.G = {k: torch.empty_like(v) for k, v in A.items() if k != "x0"}
        f32 = dict(dtype=torch.float32, device=self.dev)
        self.base = torch.empty((B, H, W, 2), **f32)
        self.pred = torch.empty((B, H, W, 2), **f32)
        self.loss_dev = torch.empty(1, **f32)
        self.wt = torch.empty(128 * 9 * 128, **i16)
        L = lib()
        need = 0
        for lvl, (ci, co) in enumerate(ENC):
            h, w = H >> lvl, W >> lvl
            need = max(need, L.lbmnn_wgrad_partials(B, h, w, ci, co), L.lbmnn_wgrad_partials(B, h, w, co, co))
        need = max(need, L.lbmnn_wgrad_partials(B, H >> 3, W >> 3, MID, MID))
        for k, (ci, co) in enumerate(DEC):
            lvl = len(DEC) - 1 - k
            h, w = H >> lvl, W >> lvl
            need = max(need, L.lbmnn_wgrad_partials(B, h, w, ci, co), L.lbmnn_wgrad_partials(B, h, w, co, co))
        self.part = torch.empty(need, **f32)
        self.hpart = torch.empty(L.lbmnn_head_partials(B, H, W, DEC[-1][1]), **f32)

    def _view(self, t, name):
        o, shape = self.offs[name]
        return t[o:o + int(np.prod(shape))]

    # -- parameters ------------------------------------------------------
    def set_params(self, params):
        import torch
        host = np.zeros(self.nparam, dtype=np.float32)
        for name, (o, shape) in self.offs.items():
            a = np.asarray(params[name], dtype=np.float32)
            if a.shape != tuple(shape):
                raise ValueError("%s: expected %s, got %s" % (name, shape, a.shape))
            host[o:o + a.size] = a.reshape(-1)
        self.w32.copy_(torch.from_numpy(host))
        _chk("lbmnn_to_bf16", lib().lbmnn_to_bf16(_p(self.w32), _p(self.w16), self.nparam, self.sp))
        self.m.zero_()
        self.v.zero_()
        self.t = 0

    def get_params(self):
        host = self.w32.cpu().numpy()
        return {name: host[o:o + int(np.prod(shape))].reshape(shape).astype(np.float64)
                for name, (o, shape) in self.offs.items()}

    def get_grads(self):
        host = self.g32.cpu().numpy()
        return {name: host[o:o + int(np.prod(shape))].reshape(shape).astype(np.float64)
                for name, (o, shape) in self.offs.items()}

    # -- layers ----------------------------------------------------------
    def _conv(self, name, x, y, relu=True):
        w = self._view(self.w16, name + ".w")
        b = self._view(self.w32, name + ".b")
        _chk("lbmnn_conv3x3", lib().lbmnn_conv3x3(
            x.ptr, x.cs, x.co, None, 0, 0, _p(w), _p(b), y.ptr, y.cs, y.co,
            x.B, x.H, x.W, x.C, y.C, int(relu), self.wrap, self.sp))

    def _conv_back(self, name, x, y, dy, dx):
        """Weight/bias gradients into g32; input gradient into dx (if any)."""
        L = lib()
        gw = self._view(self.g32, name + ".w")
        gb = self._view(self.g32, name + ".b")
        _chk("lbmnn_conv3x3_wgrad", L.lbmnn_conv3x3_wgrad(
            x.ptr, x.cs, x.co, dy.ptr, dy.cs, dy.co, y.ptr, y.cs, y.co, _p(gw), _p(gb), _p(self.part),
            x.B, x.H, x.W, x.C, y.C, self.wrap, self.sp))
        if dx is not None:
            w = self._view(self.w16, name + ".w")
            _chk("lbmnn_conv3x3_flip", L.lbmnn_conv3x3_flip(_p(w), _p(self.wt), x.C, y.C, self.sp))
            _chk("lbmnn_conv3x3", L.lbmnn_conv3x3(
                dy.ptr, dy.cs, dy.co, y.ptr, y.cs, y.co, _p(self.wt), None, dx.ptr, dx.cs, dx.co,
                x.B, x.H, x.W, y.C, x.C, 0, self.wrap, self.sp))

    def _acts(self, D):
        """Named activation windows over the buffers in D."""
        a = {}
        a["x0"] = Act(self.A["x0"], 0, IN_CH) if "x0" in D else None
        for lvl, (ci, co) in enumerate(ENC):
            cat = D["cat%d" % lvl]
            a["enc%d_a" % lvl] = Act(D["enc%d_a" % lvl], 0, co)
            a["skip%d" % lvl] = Act(cat, cat.shape[3] - co, co)
            a["up%d" % lvl] = Act(cat, 0, cat.shape[3] - co)
            a["cat%d" % lvl] = Act(cat, 0, cat.shape[3])
            a["pool%d" % lvl] = Act(D["pool%d" % lvl], 0, co)
        a["mid_a"] = Act(D["mid_a"], 0, MID)
        a["mid_b"] = Act(D["mid_b"], 0, MID)
        for k, (ci, co) in enumerate(DEC):
            lvl = len(DEC) - 1 - k
            a["dec%d_a" % lvl] = Act(D["dec%d_a" % lvl], 0, co)
            a["dec%d_b" % lvl] = Act(D["dec%d_b" % lvl], 0, co)
        return a

    # -- passes ----------------------------------------------------------
    def pack_input(self, rho, T, scalars, tc):
        """rho, T: float64 CUDA tensors [B, H, W]; scalars float64 [B, 3]."""
        _chk("lbmnn_pack_input", lib().lbmnn_pack_input(
            _p(rho), _p(T), _p(scalars), float(tc), _floats(NORM_SHIFT), _floats(NORM_SCALE),
            _p(self.A["x0"]), _p(self.base), self.B, self.H, self.W, self.sp))

    def pack_target(self, rho, T, tc, out):
        _chk("lbmnn_pack_target", lib().lbmnn_pack_target(
            _p(rho), _p(T), float(tc), _floats(NORM_SHIFT), _floats(NORM_SCALE), _p(out),
            self.B, self.H, self.W, self.sp))

    def forward(self):
        """Network output (normalised rho, T) for the packed input into
        self.pred (FP32 [B, H, W, 2])."""
        L = lib()
        a = self._acts(self.A)
        h = a["x0"]
        for lvl in range(len(ENC)):
            self._conv("enc%d_a" % lvl, h, a["enc%d_a" % lvl])
            self._conv("enc%d_b" % lvl, a["enc%d_a" % lvl], a["skip%d" % lvl])
            s, p = a["skip%d" % lvl], a["pool%d" % lvl]
            _chk("lbmnn_pool2", L.lbmnn_pool2(s.ptr, s.cs, s.co, p.ptr, p.cs, p.co, s.B, s.H, s.W, s.C, self.sp))
            h = p
        self._conv("mid_a", h, a["mid_a"])
        self._conv("mid_b", a["mid_a"], a["mid_b"])
        h = a["mid_b"]
        for lvl in reversed(range(len(ENC))):
            u = a["up%d" % lvl]
            _chk("lbmnn_up2", L.lbmnn_up2(h.ptr, h.cs, h.co, u.ptr, u.cs, u.co, h.B, h.H, h.W, h.C, self.sp))
            self._conv("dec%d_a" % lvl, a["cat%d" % lvl], a["dec%d_a" % lvl])
            self._conv("dec%d_b" % lvl, a["dec%d_a" % lvl], a["dec%d_b" % lvl])
            h = a["dec%d_b" % lvl]
        wh, bh = self._view(self.w32, "head.w"), self._view(self.w32, "head.b")
        _chk("lbmnn_head", L.lbmnn_head(h.ptr, h.cs, h.co, _p(self.base), _p(wh), _p(bh), _p(self.pred),
                                        self.B, self.H, self.W, h.C, self.sp))
        return self.pred

    def backward(self, target):
        """Loss (into self.loss_dev) and every parameter gradient (into
        self.g32) for the last forward pass against `target` (FP32
        [B, H, W, 2], normalised)."""
        L = lib()
        a = self._acts(self.A)
        d = self._acts(self.G)
        f, df = a["dec0_b"], d["dec0_b"]
        wh, bh = self._view(self.w32, "head.w"), self._view(self.w32, "head.b")
        gwh, gbh = self._view(self.g32, "head.w"), self._view(self.g32, "head.b")
        _chk("lbmnn_head_loss", L.lbmnn_head_loss(
            f.ptr, f.cs, f.co, _p(self.base), _p(wh), _p(bh), _p(target), _p(self.loss_dev), _p(gwh),
            _p(gbh), df.ptr, df.cs, df.co, _p(self.hpart), self.B, self.H, self.W, f.C, self.sp))
        dh = df
        for lvl in range(len(ENC)):
            self._conv_back("dec%d_b" % lvl, a["dec%d_a" % lvl], a["dec%d_b" % lvl], dh, d["dec%d_a" % lvl])
            self._conv_back("dec%d_a" % lvl, a["cat%d" % lvl], a["dec%d_a" % lvl], d["dec%d_a" % lvl],
                            d["cat%d" % lvl])
            du = d["up%d" % lvl]
            nxt = d["dec%d_b" % (lvl + 1)] if lvl + 1 < len(ENC) else d["mid_b"]
            _chk("lbmnn_up2_back", L.lbmnn_up2_back(du.ptr, du.cs, du.co, nxt.ptr, nxt.cs, nxt.co, nxt.B,
                                                    nxt.H, nxt.W, nxt.C, self.sp))
            dh = nxt
        self._conv_back("mid_b", a["mid_a"], a["mid_b"], dh, d["mid_a"])
        top = len(ENC) - 1
        self._conv_back("mid_a", a["pool%d" % top], a["mid_a"], d["mid_a"], d["pool%d" % top])
        for lvl in reversed(range(len(ENC))):
            dp, ds = d["pool%d" % lvl], d["skip%d" % lvl]
            _chk("lbmnn_pool2_back", L.lbmnn_pool2_back(dp.ptr, dp.cs, dp.co, ds.ptr, ds.cs, ds.co, ds.B, ds.H,
                                                        ds.W, ds.C, self.sp))
            self._conv_back("enc%d_b" % lvl, a["enc%d_a" % lvl], a["skip%d" % lvl], ds, d["enc%d_a" % lvl])
            x_in = a["pool%d" % (lvl - 1)] if lvl > 0 else a["x0"]
            dx = d["pool%d" % (lvl - 1)] if lvl > 0 else None
            self._conv_back("enc%d_a" % lvl, x_in, a["enc%d_a" % lvl], d["enc%d_a" % lvl], dx)
        return self.loss_dev

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.t += 1
        _chk("lbmnn_adam", lib().lbmnn_adam(_p(self.w32), _p(self.w16), _p(self.g32), _p(self.m), _p(self.v),
                                            self.nparam, lr, beta1, beta2, eps, self.t, self.sp))

    def unpack(self, rho, T, tc):
        """self.pred back to FP64 fields rho, T (CUDA tensors [B, H, W])."""
        _chk("lbmnn_unpack_output", lib().lbmnn_unpack_output(
            _p(self.pred), float(tc), _floats(NORM_SHIFT), _floats(NORM_SCALE), _p(rho), _p(T),
            self.B, self.H, self.W, self.sp))
