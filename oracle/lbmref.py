"""ctypes wrapper of the FP64 oracle (test infrastructure only).

Parameters are passed as a plain dict (the same dict the HIP binding
takes); this module fills the oracle's own C struct from it.
"""
import ctypes
import os

import numpy as np

from . import build as _build

PLAIN = 0
CORRECTED = 1
FD_RK2 = 2

_EOS = {"cs": 0, "ideal": 1}
_THERMAL = {"dirichlet": 0, "adiabatic": 1}


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("tau_f", ctypes.c_double), ("tau_g", ctypes.c_double),
        ("G", ctypes.c_double), ("beta", ctypes.c_double),
        ("eos", ctypes.c_int), ("a", ctypes.c_double), ("b", ctypes.c_double),
        ("R", ctypes.c_double),
        ("eos_fixed_T", ctypes.c_int), ("T_eos", ctypes.c_double),
        ("cv", ctypes.c_double),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double),
        ("wall_x", ctypes.c_int), ("wall_y", ctypes.c_int),
        ("thermal_left", ctypes.c_int), ("thermal_right", ctypes.c_int),
        ("thermal_bottom", ctypes.c_int), ("thermal_top", ctypes.c_int),
        ("T_left", ctypes.c_double), ("T_right", ctypes.c_double),
        ("T_bottom", ctypes.c_double), ("T_top", ctypes.c_double),
        ("psi_policy", ctypes.c_int),
        ("u_in", ctypes.c_double),
        ("rho_out", ctypes.c_double),
        ("phi_divu", ctypes.c_int),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.lbmref_create.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(ctypes.c_void_p)]
        L.lbmref_destroy.argtypes = [ctypes.c_void_p]
        L.lbmref_init_fields.argtypes = [ctypes.c_void_p, dp, dp, dp, dp]
        L.lbmref_step.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
        L.lbmref_moments.argtypes = [ctypes.c_void_p, dp, dp, dp, dp]
        L.lbmref_totals.argtypes = [ctypes.c_void_p, dp]
        L.lbmref_get_state.argtypes = [ctypes.c_void_p, dp, dp]
        L.lbmref_set_state.argtypes = [ctypes.c_void_p, dp, dp]
        L.lbmref_force.argtypes = [ctypes.c_void_p, dp, dp]
        L.lbmref_psi.argtypes = [ctypes.c_void_p, dp, dp]
        L.lbmref_velocities.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), dp]
        L.lbmref_feq.argtypes = [ctypes.c_double] * 3 + [dp]
        L.lbmref_guo.argtypes = [ctypes.c_double] * 5 + [dp]
        L.lbmref_corr.argtypes = [ctypes.c_double] * 4 + [dp]
        L.lbmref_pressure.argtypes = [ctypes.POINTER(_Params), ctypes.c_double, ctypes.c_double]
        L.lbmref_pressure.restype = ctypes.c_double
        L.lbmref_sc_force_field.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                            dp, dp, dp, dp]
        _lib = L
    return _lib


def make_params(cfg):
    """Oracle parameter struct from a parameter dict (missing keys take
    the defaults of the static-droplet workload's model)."""
    p = _Params()
    p.nx = int(cfg["nx"])
    p.ny = int(cfg["ny"])
    p.tau_f = float(cfg.get("tau_f", 1.0))
    p.tau_g = float(cfg.get("tau_g", 0.8))
    p.G = float(cfg.get("G", -1.0))
    p.beta = float(cfg.get("beta", 1.0))
    p.eos = _EOS[cfg.get("eos", "cs")]
    p.a = float(cfg.get("a", 1.0))
    p.b = float(cfg.get("b", 4.0))
    p.R = float(cfg.get("R", 1.0))
    p.eos_fixed_T = int(bool(cfg.get("eos_fixed_T", False)))
    p.T_eos = float(cfg.get("T_eos", 0.0))
    p.cv = float(cfg.get("cv", 1.0))
    p.gx = float(cfg.get("gx", 0.0))
    p.gy = float(cfg.get("gy", 0.0))
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
    return p


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a, n):
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
    assert a.size == n, (a.size, n)
    return a


class Oracle:
    """One lattice held by the FP64 oracle."""

    def __init__(self, cfg):
        self.cfg = dict(cfg)
        self.nx, self.ny = int(cfg["nx"]), int(cfg["ny"])
        self._p = make_params(cfg)
        h = ctypes.c_void_p()
        rc = lib().lbmref_create(ctypes.byref(self._p), ctypes.byref(h))
        if rc != 0:
            raise ValueError("lbmref_create failed with status %d" % rc)
        self._h = h

    def close(self):
        if self._h:
            lib().lbmref_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n(self):
        return self.nx * self.ny

    def init_fields(self, rho, T, ux=None, uy=None):
        n = self.n
        r = _f64(rho, n)
        t = _f64(T, n)
        u = _f64(ux, n) if ux is not None else None
        v = _f64(uy, n) if uy is not None else None
        rc = lib().lbmref_init_fields(self._h, _dp(r), _dp(u) if u is not None else None,
                                      _dp(v) if v is not None else None, _dp(t))
        if rc != 0:
            raise RuntimeError("lbmref_init_fields: %d" % rc)

    def init_fields_physical(self, rho, T, ux=None, uy=None):
        """Equilibrium start whose velocity in the forcing scheme of Eq. (1)
        (Sec. II: u = (j + F/2)/rho) is the given u: f = f_eq(rho, u -
        F/(2 rho)) and g = cv T f.  F is the total force of the given rho
        and T (psi of Eq. (2) or (4) depends on them alone, and so does the
        body force), read from a first equilibrium start."""
        r = _f64(rho, self.n).reshape(self.ny, self.nx)
        self.init_fields(r, T)
        Fx, Fy = self.force()
        u = 0.0 if ux is None else _f64(ux, self.n).reshape(self.ny, self.nx)
        v = 0.0 if uy is None else _f64(uy, self.n).reshape(self.ny, self.nx)
        self.init_fields(r, T, u - 0.5 * Fx / r, v - 0.5 * Fy / r)

    def step(self, n, treatment):
        return lib().lbmref_step(self._h, int(n), int(treatment))

    def moments(self):
        n = self.n
        out = [np.empty(n) for _ in range(4)]
        rc = lib().lbmref_moments(self._h, *[_dp(a) for a in out])
        if rc != 0:
            raise RuntimeError("lbmref_moments: %d" % rc)
        return [a.reshape(self.ny, self.nx) for a in out]

    def totals(self):
        out = np.zeros(8)
        rc = lib().lbmref_totals(self._h, _dp(out))
        if rc != 0:
            raise RuntimeError("lbmref_totals: %d" % rc)
        return out

    def get_state(self):
        f = np.empty(9 * self.n)
        g = np.empty(9 * self.n)
        rc = lib().lbmref_get_state(self._h, _dp(f), _dp(g))
        if rc != 0:
            raise RuntimeError("lbmref_get_state: %d" % rc)
        return f.reshape(9, self.ny, self.nx), g.reshape(9, self.ny, self.nx)

    def set_state(self, f, g):
        f = _f64(f, 9 * self.n)
        g = _f64(g, 9 * self.n)
        rc = lib().lbmref_set_state(self._h, _dp(f), _dp(g))
        if rc != 0:
            raise RuntimeError("lbmref_set_state: %d" % rc)

    def force(self):
        Fx = np.empty(self.n)
        Fy = np.empty(self.n)
        rc = lib().lbmref_force(self._h, _dp(Fx), _dp(Fy))
        if rc != 0:
            raise RuntimeError("lbmref_force: %d" % rc)
        return Fx.reshape(self.ny, self.nx), Fy.reshape(self.ny, self.nx)

    def psi(self):
        a = np.empty(self.n)
        b = np.empty(self.n)
        rc = lib().lbmref_psi(self._h, _dp(a), _dp(b))
        if rc != 0:
            raise RuntimeError("lbmref_psi: %d" % rc)
        return a.reshape(self.ny, self.nx), b.reshape(self.ny, self.nx)


def velocities():
    ex = (ctypes.c_int * 9)()
    ey = (ctypes.c_int * 9)()
    w = np.empty(9)
    lib().lbmref_velocities(ex, ey, _dp(w))
    return np.array(list(ex)), np.array(list(ey)), w


def feq(rho, ux, uy):
    out = np.empty(9)
    lib().lbmref_feq(rho, ux, uy, _dp(out))
    return out


def guo(tau_f, ux, uy, Fx, Fy):
    out = np.empty(9)
    lib().lbmref_guo(tau_f, ux, uy, Fx, Fy, _dp(out))
    return out


def corr(tau_g, cvT, Fx, Fy):
    out = np.empty(9)
    lib().lbmref_corr(tau_g, cvT, Fx, Fy, _dp(out))
    return out


def pressure(cfg, rho, T):
    p = make_params(dict(cfg, nx=1, ny=1))
    return lib().lbmref_pressure(ctypes.byref(p), float(rho), float(T))


def sc_force_field(psi, psi2, G, beta=1.0, wall_x=False, wall_y=False):
    psi = np.ascontiguousarray(psi, dtype=np.float64)
    psi2 = np.ascontiguousarray(psi2, dtype=np.float64)
    ny, nx = psi.shape
    Fx = np.empty((ny, nx))
    Fy = np.empty((ny, nx))
    lib().lbmref_sc_force_field(nx, ny, G, beta, int(wall_x), int(wall_y), _dp(psi), _dp(psi2),
                                _dp(Fx), _dp(Fy))
    return Fx, Fy
