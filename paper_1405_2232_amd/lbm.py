"""Python binding of liblbm (include/lbm.h): argument marshalling only.

Every step of the method runs in the HIP library; PyTorch supplies the
device workspace (a uint8 tensor) and the stream.  If the library is not
built, loading raises: there is no CPU fallback.
"""
import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "lbm.h")

OK, EINVAL, ENOMEM, EDEVICE, ENONFINITE, EDOMAIN, ESTATE = 0, -1, -2, -3, -4, -5, -6
PLAIN, CORRECTED, FD_RK2 = 0, 1, 2
FP64, FP32_DEV, FP32_LOCAL = 0, 1, 2
_EOS = {"cs": 0, "ideal": 1}
_THERMAL = {"dirichlet": 0, "adiabatic": 1}
_PREC = {"fp64": FP64, "fp32dev": FP32_DEV, "fp32local": FP32_LOCAL,
         FP64: FP64, FP32_DEV: FP32_DEV, FP32_LOCAL: FP32_LOCAL}


class LbmError(RuntimeError):
    def __init__(self, fn, status):
        self.status = status
        msg = lib().lbm_strerror(status).decode() if _lib is not None else str(status)
        super().__init__("%s failed: %s (%d)" % (fn, msg, status))


class Params(ctypes.Structure):
    """Mirror of lbm_params."""
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("tau_f", ctypes.c_double), ("tau_g", ctypes.c_double),
        ("G", ctypes.c_double), ("beta", ctypes.c_double),
        ("eos", ctypes.c_int), ("a", ctypes.c_double), ("b", ctypes.c_double), ("R", ctypes.c_double),
        ("eos_fixed_T", ctypes.c_int), ("T_eos", ctypes.c_double),
        ("cv", ctypes.c_double),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double),
        ("wall_x", ctypes.c_int), ("wall_y", ctypes.c_int),
        ("thermal_left", ctypes.c_int), ("thermal_right", ctypes.c_int),
        ("thermal_bottom", ctypes.c_int), ("thermal_top", ctypes.c_int),
        ("T_left", ctypes.c_double), ("T_right", ctypes.c_double),
        ("T_bottom", ctypes.c_double), ("T_top", ctypes.c_double),
        ("psi_policy", ctypes.c_int),
        ("precision", ctypes.c_int), ("rho_ref", ctypes.c_double), ("T_ref", ctypes.c_double),
        ("u_in", ctypes.c_double), ("rho_out", ctypes.c_double),
        ("phi_divu", ctypes.c_int),
    ]


_lib = None


def header_functions(header=HEADER):
    """Names of the functions a header under include/ declares."""
    txt = open(header).read()
    return sorted(set(re.findall(r"^\s*(?:int|size_t|const char|void)\s*\*?\s*(lbm\w*_\w+)\s*\(", txt, re.M)))


def lib():
    """Load liblbm.so (building it in-tree first if nothing is built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, i, sz = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_size_t
        P = ctypes.POINTER(Params)
        sig = {
            "lbm_workspace_bytes": [P, ctypes.POINTER(sz)],
            "lbm_create": [P, vp, sz, vp, ctypes.POINTER(vp)],
            "lbm_init_fields": [vp, dp, dp, dp, dp],
            "lbm_init_fields_physical": [vp, dp, dp, dp, dp],
            "lbm_step": [vp, i, i],
            "lbm_set_check_interval": [vp, i],
            "lbm_sync": [vp],
            "lbm_moments": [vp, dp, dp, dp, dp],
            "lbm_moments_device": [vp, vp, vp, vp, vp],
            "lbm_totals": [vp, dp],
            "lbm_totals_noalloc": [vp, dp],
            "lbm_step_residual": [vp, i, dp],
            "lbm_get_state": [vp, dp],
            "lbm_set_state": [vp, dp],
            "lbm_save": [vp, ctypes.c_char_p],
            "lbm_load": [vp, ctypes.c_char_p],
            "lbm_set_tiling": [vp, i, i],
            "lbm_get_tiling": [vp, ctypes.POINTER(i), ctypes.POINTER(i)],
            "lbm_set_step_pairing": [vp, i, i],
            "lbm_get_step_pairing": [vp, ctypes.POINTER(i), ctypes.POINTER(i)],
            "lbm_destroy": [vp],
            "lbm_copy_probe": [vp, vp, sz, vp],
            "lbm_batch_workspace_bytes": [i, P, ctypes.POINTER(sz)],
            "lbm_batch_create": [i, P, vp, sz, vp, ctypes.POINTER(vp)],
            "lbm_batch_lattice": [vp, i, ctypes.POINTER(vp)],
            "lbm_batch_init_fields": [vp, i, dp, dp, dp, dp],
            "lbm_batch_init_fields_physical": [vp, i, dp, dp, dp, dp],
            "lbm_batch_moments": [vp, i, dp, dp, dp, dp],
            "lbm_batch_step": [vp, i, i],
            "lbm_batch_step_residuals": [vp, i, dp, ctypes.POINTER(i)],
            "lbm_batch_set_active": [vp, ctypes.POINTER(i)],
            "lbm_batch_set_tiling": [vp, i, i],
            "lbm_batch_get_tiling": [vp, ctypes.POINTER(i), ctypes.POINTER(i)],
            "lbm_batch_use_graph": [vp, i],
            "lbm_batch_set_step_pairing": [vp, i, i],
            "lbm_batch_get_step_pairing": [vp, ctypes.POINTER(i), ctypes.POINTER(i)],
            "lbm_batch_sync": [vp],
            "lbm_batch_destroy": [vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.lbm_strerror.argtypes = [ctypes.c_int]
        L.lbm_strerror.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _chk(fn, rc):
    if rc != OK:
        raise LbmError(fn, rc)
    return rc


def make_params(cfg, precision="fp64", rho_ref=None, T_ref=None):
    """lbm_params from a parameter dict (the same dict the oracle takes)."""
    p = Params()
    p.nx, p.ny = int(cfg["nx"]), int(cfg["ny"])
    p.tau_f = float(cfg.get("tau_f", 1.0))
    p.tau_g = float(cfg.get("tau_g", 0.8))
    p.G = float(cfg.get("G", -1.0))
    p.beta = float(cfg.get("beta", 1.0))
    p.eos = _EOS[cfg.get("eos", "cs")]
    p.a, p.b, p.R = float(cfg.get("a", 1.0)), float(cfg.get("b", 4.0)), float(cfg.get("R", 1.0))
    p.eos_fixed_T = int(bool(cfg.get("eos_fixed_T", False)))
    p.T_eos = float(cfg.get("T_eos", 0.0))
    p.cv = float(cfg.get("cv", 1.0))
    p.gx, p.gy = float(cfg.get("gx", 0.0)), float(cfg.get("gy", 0.0))
    wx = cfg.get("wall_x", False)
    p.wall_x = 2 if (wx == "open" or (not isinstance(wx, bool) and wx == 2)) else int(bool(wx))
    p.wall_y = int(bool(cfg.get("wall_y", False)))
    for side in ("left", "right", "bottom", "top"):
        setattr(p, "thermal_" + side, _THERMAL[cfg.get("thermal_" + side, "dirichlet")])
        setattr(p, "T_" + side, float(cfg.get("T_" + side, 0.0)))
    p.psi_policy = int(cfg.get("psi_policy", 0))
    p.u_in = float(cfg.get("u_in", 0.0))
    p.rho_out = float(cfg.get("rho_out", 1.0))
    p.phi_divu = int(bool(cfg.get("phi_divu", False)))
    p.precision = _PREC[precision]
    p.rho_ref = float(rho_ref if rho_ref is not None else cfg.get("rho_ref", 0.0))
    p.T_ref = float(T_ref if T_ref is not None else cfg.get("T_ref", 0.0))
    return p


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _host(a, n):
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
    if a.size != n:
        raise ValueError("expected %d values, got %d" % (n, a.size))
    return a


def workspace_bytes(cfg, precision="fp64", rho_ref=None, T_ref=None):
    p = make_params(cfg, precision, rho_ref, T_ref)
    n = ctypes.c_size_t()
    _chk("lbm_workspace_bytes", lib().lbm_workspace_bytes(ctypes.byref(p), ctypes.byref(n)))
    return n.value


class _HandleOps:
    """Calls on one lattice handle (owned by a Lattice or by a Batch)."""

    @property
    def n(self):
        return self.nx * self.ny

    @property
    def handle(self):
        return self._h

    def _init(self, rho, T, ux=None, uy=None, physical=False):
        n = self.n
        r, t = _host(rho, n), _host(T, n)
        u = _host(ux, n) if ux is not None else None
        v = _host(uy, n) if uy is not None else None
        name = "lbm_init_fields_physical" if physical else "lbm_init_fields"
        _chk(name, getattr(lib(), name)(self._h, _dp(r), _dp(u) if u is not None else None,
                                        _dp(v) if v is not None else None, _dp(t)))

    def step(self, n, treatment, check=True):
        rc = lib().lbm_step(self._h, int(n), int(treatment))
        if check:
            _chk("lbm_step", rc)
        return rc

    def set_check_interval(self, k):
        _chk("lbm_set_check_interval", lib().lbm_set_check_interval(self._h, int(k)))

    def sync(self):
        return lib().lbm_sync(self._h)

    def moments(self, check=True):
        out = [np.empty(self.n) for _ in range(4)]
        rc = lib().lbm_moments(self._h, *[_dp(a) for a in out])
        if check:
            _chk("lbm_moments", rc)
        return [a.reshape(self.ny, self.nx) for a in out]

    def moments_device(self, rho=None, ux=None, uy=None, T=None):
        """Write moments into caller-owned torch float64 CUDA tensors (stream-ordered)."""
        ptr = [ctypes.c_void_p(t.data_ptr()) if t is not None else None for t in (rho, ux, uy, T)]
        _chk("lbm_moments_device", lib().lbm_moments_device(self._h, *ptr))

    def totals(self):
        out = np.zeros(8)
        _chk("lbm_totals", lib().lbm_totals(self._h, _dp(out)))
        return out

    def totals_noalloc(self):
        """lbm_totals_noalloc: the same totals with the library's static
        scratch array (no workspace scratch)."""
        out = np.zeros(8)
        _chk("lbm_totals_noalloc", lib().lbm_totals_noalloc(self._h, _dp(out)))
        return out

    def step_residual(self, treatment):
        r = ctypes.c_double()
        _chk("lbm_step_residual", lib().lbm_step_residual(self._h, int(treatment), ctypes.byref(r)))
        return r.value

    def get_state(self):
        s = np.empty(18 * self.n)
        _chk("lbm_get_state", lib().lbm_get_state(self._h, _dp(s)))
        return s.reshape(18, self.ny, self.nx)

    def set_state(self, state):
        s = _host(state, 18 * self.n)
        _chk("lbm_set_state", lib().lbm_set_state(self._h, _dp(s)))

    def save(self, path):
        _chk("lbm_save", lib().lbm_save(self._h, os.fsencode(path)))

    def load(self, path):
        _chk("lbm_load", lib().lbm_load(self._h, os.fsencode(path)))

    def set_tiling(self, bx, rows):
        _chk("lbm_set_tiling", lib().lbm_set_tiling(self._h, int(bx), int(rows)))

    def get_tiling(self):
        a, b = ctypes.c_int(), ctypes.c_int()
        _chk("lbm_get_tiling", lib().lbm_get_tiling(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def set_step_pairing(self, on, rows=0):
        _chk("lbm_set_step_pairing", lib().lbm_set_step_pairing(self._h, int(bool(on)), int(rows)))

    def get_step_pairing(self):
        """(pairing used by step(), rows per block of the two-step kernel)"""
        a, b = ctypes.c_int(), ctypes.c_int()
        _chk("lbm_get_step_pairing", lib().lbm_get_step_pairing(self._h, ctypes.byref(a), ctypes.byref(b)))
        return bool(a.value), b.value


class Lattice(_HandleOps):
    """One lattice on the GPU.  `precision` is "fp64", "fp32dev" (global
    deviation shifts) or "fp32local" (per-node density shift); rho_ref and
    T_ref default to the mean initial density and temperature (set at
    init_fields unless given here)."""

    def __init__(self, cfg, precision="fp64", rho_ref=None, T_ref=None, device=None, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("liblbm needs a ROCm GPU; none is visible")
        self.cfg = dict(cfg)
        self.nx, self.ny = int(cfg["nx"]), int(cfg["ny"])
        self.precision = precision
        self._rho_ref, self._T_ref = rho_ref, T_ref
        self.device = torch.device(device if device is not None else "cuda")
        self._stream = stream
        self._h = None
        self.ws = None

    # creation is deferred to init_fields when the deviation shifts come
    # from the initial fields
    def _create(self, rho_ref, T_ref):
        import torch
        self.close()
        self._p = make_params(self.cfg, self.precision, rho_ref, T_ref)
        n = ctypes.c_size_t()
        _chk("lbm_workspace_bytes", lib().lbm_workspace_bytes(ctypes.byref(self._p), ctypes.byref(n)))
        self.ws = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        s = self._stream if self._stream is not None else torch.cuda.current_stream(self.device)
        self.stream = s
        h = ctypes.c_void_p()
        _chk("lbm_create", lib().lbm_create(ctypes.byref(self._p), ctypes.c_void_p(self.ws.data_ptr()),
                                            n.value, ctypes.c_void_p(s.cuda_stream), ctypes.byref(h)))
        self._h = h

    def init_fields(self, rho, T, ux=None, uy=None, physical=False):
        """Equilibrium distributions of rho, u, T; `physical` stores the
        momentum rho u - F/2 so that the reported velocity (j + F/2)/rho is
        u (lbm_init_fields_physical)."""
        r, t = _host(rho, self.n), _host(T, self.n)
        rho_ref = self._rho_ref if self._rho_ref is not None else float(r.mean())
        T_ref = self._T_ref if self._T_ref is not None else float(t.mean())
        if self._h is None or (self.precision != "fp64" and
                               (rho_ref != self._p.rho_ref or T_ref != self._p.T_ref)):
            self._create(rho_ref, T_ref)
        self._init(r, t, ux, uy, physical)

    def close(self):
        if self._h is not None:
            lib().lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _Member(_HandleOps):
    def __init__(self, batch, i, h, nx, ny):
        self._batch = batch  # keeps the batch (and its workspace) alive
        self.i = i
        self._h = h
        self.nx, self.ny = nx, ny

    def init_fields(self, rho, T, ux=None, uy=None, physical=False):
        self._init(rho, T, ux, uy, physical)


class Batch:
    """Many lattices stepped together.  `cfgs` is a list of parameter dicts
    (sizes and parameters may differ); `refs` optionally gives (rho_ref,
    T_ref) per lattice for the FP32 storage forms."""

    def __init__(self, cfgs, precision="fp64", refs=None, device=None, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("liblbm needs a ROCm GPU; none is visible")
        self.count = len(cfgs)
        refs = refs if refs is not None else [(None, None)] * self.count
        P = (Params * self.count)()
        for i, c in enumerate(cfgs):
            P[i] = make_params(c, precision, refs[i][0], refs[i][1])
        self._P = P
        n = ctypes.c_size_t()
        _chk("lbm_batch_workspace_bytes", lib().lbm_batch_workspace_bytes(self.count, P, ctypes.byref(n)))
        dev = torch.device(device if device is not None else "cuda")
        self.ws = torch.empty(n.value, dtype=torch.uint8, device=dev)
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        self.stream = s
        h = ctypes.c_void_p()
        _chk("lbm_batch_create", lib().lbm_batch_create(self.count, P, ctypes.c_void_p(self.ws.data_ptr()),
                                                        n.value, ctypes.c_void_p(s.cuda_stream),
                                                        ctypes.byref(h)))
        self._h = h
        self.members = []
        for i, c in enumerate(cfgs):
            m = ctypes.c_void_p()
            _chk("lbm_batch_lattice", lib().lbm_batch_lattice(h, i, ctypes.byref(m)))
            self.members.append(_Member(self, i, m, int(c["nx"]), int(c["ny"])))

    def __getitem__(self, i):
        return self.members[i]

    def __len__(self):
        return self.count

    def step(self, n, treatment):
        _chk("lbm_batch_step", lib().lbm_batch_step(self._h, int(n), int(treatment)))

    def step_residuals(self, treatment):
        """(residuals, statuses) of every lattice after one batch step
        (lbm_batch_step_residuals; inactive lattices: -1 and OK)."""
        r = np.empty(self.count)
        s = (ctypes.c_int * self.count)()
        _chk("lbm_batch_step_residuals", lib().lbm_batch_step_residuals(self._h, int(treatment), _dp(r), s))
        return r, list(s)

    def set_active(self, active=None):
        if active is None:
            _chk("lbm_batch_set_active", lib().lbm_batch_set_active(self._h, None))
        else:
            a = (ctypes.c_int * self.count)(*[int(bool(x)) for x in active])
            _chk("lbm_batch_set_active", lib().lbm_batch_set_active(self._h, a))

    def set_tiling(self, bx, rows):
        _chk("lbm_batch_set_tiling", lib().lbm_batch_set_tiling(self._h, int(bx), int(rows)))

    def get_tiling(self):
        a, b = ctypes.c_int(), ctypes.c_int()
        _chk("lbm_batch_get_tiling", lib().lbm_batch_get_tiling(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def use_graph(self, k):
        _chk("lbm_batch_use_graph", lib().lbm_batch_use_graph(self._h, int(k)))

    def set_step_pairing(self, on, rows=0):
        _chk("lbm_batch_set_step_pairing",
             lib().lbm_batch_set_step_pairing(self._h, int(bool(on)), int(rows)))

    def get_step_pairing(self):
        """(pairing used by step(), band height of the two-step tiles)"""
        a, b = ctypes.c_int(), ctypes.c_int()
        _chk("lbm_batch_get_step_pairing",
             lib().lbm_batch_get_step_pairing(self._h, ctypes.byref(a), ctypes.byref(b)))
        return bool(a.value), b.value

    def sync(self):
        return lib().lbm_batch_sync(self._h)

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().lbm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def copy_probe(dst, src, stream=None):
    """Plain streaming copy of a torch CUDA tensor (bandwidth ceiling)."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream(dst.device)
    nbytes = src.numel() * src.element_size()
    _chk("lbm_copy_probe", lib().lbm_copy_probe(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()),
                                                nbytes, ctypes.c_void_p(s.cuda_stream)))
