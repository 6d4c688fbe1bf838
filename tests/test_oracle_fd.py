"""Pins of the oracle's third temperature treatment: the finite-difference
solution of Eq. (26) with the Runge-Kutta scheme of Eq. (27).

- One step agrees with an independent NumPy evaluation of the same
  isotropic central differences and stages (brute force, small lattice).
- A linear conduction profile between Dirichlet walls is a fixed point, and
  a uniform initial temperature relaxes to it.
- A Gaussian diffuses at chi = (tau_g - 1/2) c_s^2 with second-order error.
- A uniform temperature stays uniform around a droplet (no force enters
  Eq. (26)), and mass is conserved.
- The paper's comparison (Sec. III): in a heated single-phase cavity the
  finite-difference and corrected LB temperatures nearly coincide, while
  the plain LB equation departs from both.
"""
import math

import numpy as np
import pytest

from oracle import CORRECTED, FD_RK2, PLAIN, Oracle
from paper_1405_2232_amd import inputs

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
WSC = np.array([0, 1 / 3, 1 / 3, 1 / 3, 1 / 3, 1 / 12, 1 / 12, 1 / 12, 1 / 12])


def _numpy_fd_step(T, rho, ux, uy, tau_g, cv=1.0):
    """Heun step of dT/dt = -u.grad T + div(lambda grad T)/(rho cv) on a
    periodic lattice, written with np.roll (no shared code with the C
    oracle)."""
    lam = (tau_g - 0.5) * cv * rho / 3.0

    def K(T):
        gx = sum(WSC[i] * EX[i] * np.roll(T, (-EY[i], -EX[i]), axis=(0, 1)) for i in range(1, 9))
        gy = sum(WSC[i] * EY[i] * np.roll(T, (-EY[i], -EX[i]), axis=(0, 1)) for i in range(1, 9))
        lx = sum(WSC[i] * EX[i] * np.roll(lam, (-EY[i], -EX[i]), axis=(0, 1)) for i in range(1, 9))
        ly = sum(WSC[i] * EY[i] * np.roll(lam, (-EY[i], -EX[i]), axis=(0, 1)) for i in range(1, 9))
        lap = sum(2 * WSC[i] * (np.roll(T, (-EY[i], -EX[i]), axis=(0, 1)) - T) for i in range(1, 9))
        return -(ux * gx + uy * gy) + (lam * lap + lx * gx + ly * gy) / (rho * cv)

    k1 = K(T)
    k2 = K(T + k1)
    return T + 0.5 * (k1 + k2)


def test_one_step_matches_independent_numpy():
    p, rho, T = inputs.static_droplet(nx=20, ny=16, radius=5, seed=3)
    p["tau_g"] = 0.9
    o = Oracle(p)
    o.init_fields(rho, T)
    r0, ux, uy, T0 = o.moments()
    assert o.step(1, FD_RK2) == 0
    T1 = o.moments()[3]
    want = _numpy_fd_step(T0, r0, ux, uy, 0.9)
    assert np.abs(T1 - want).max() < 1e-15 * 50


@pytest.mark.parametrize("tau_g", [0.6, 1.0])
def test_linear_conduction_is_a_fixed_point_and_the_limit(tau_g):
    ny = 16
    p = inputs.base_params(2, ny, 1.0, tau_g=tau_g)
    p.update(G=0.0, wall_y=True, thermal_bottom="dirichlet", thermal_top="dirichlet",
             T_bottom=0.9, T_top=1.1)
    y = np.arange(ny)
    lin = np.tile((0.9 + 0.2 * (y + 0.5) / ny)[:, None], (1, 2))
    o = Oracle(p)
    o.init_fields(np.ones((ny, 2)), lin)
    o.step(200, FD_RK2)
    assert np.abs(o.moments()[3] - lin).max() < 1e-14
    o = Oracle(p)
    o.init_fields(np.ones((ny, 2)), np.ones((ny, 2)))
    chi = (tau_g - 0.5) / 3
    o.step(int(40 / (chi * (math.pi / ny) ** 2)), FD_RK2)
    assert np.abs(o.moments()[3] - lin).max() < 1e-12


def _gauss_fd(n, sigma0, tau_g, t):
    p = inputs.base_params(n, n, 1.0, tau_g=tau_g)
    p["G"] = 0.0
    c = n / 2.0
    y, x = np.mgrid[0:n, 0:n]
    r2 = (x - c) ** 2 + (y - c) ** 2
    A = 0.01
    T0 = 1.0 + A * np.exp(-r2 / (2 * sigma0 ** 2))
    o = Oracle(p)
    o.init_fields(np.ones((n, n)), T0)
    o.step(t, FD_RK2)
    chi = (tau_g - 0.5) / 3
    s2 = sigma0 ** 2 + 2 * chi * t
    exact = 1.0 + A * sigma0 ** 2 / s2 * np.exp(-r2 / (2 * s2))
    return np.abs(o.moments()[3] - exact).max() / A


def test_gaussian_diffusion_second_order():
    tau_g = 0.8
    chi = (tau_g - 0.5) / 3
    t1 = int(round(16.0 / chi))
    e1 = _gauss_fd(64, 4.0, tau_g, t1)
    e2 = _gauss_fd(128, 8.0, tau_g, 4 * t1)
    order = math.log(e1 / e2, 2)
    assert e2 < 1e-3
    assert 1.8 < order < 2.2, (e1, e2, order)


def test_uniform_temperature_stays_uniform_around_a_droplet():
    p, rho, _ = inputs.static_droplet(nx=40, ny=40, radius=10, seed=4)
    T = np.full(rho.shape, 0.85 * inputs.cs_tc())
    o = Oracle(p)
    o.init_fields(rho, T)
    m0 = o.totals()[0]
    assert o.step(300, FD_RK2) == 0
    Tn = o.moments()[3]
    assert np.abs(Tn - T).max() < 1e-15 * 10
    assert abs(o.totals()[0] - m0) < 1e-13 * m0


def _cavity(n, Ra):
    Th, Tl, mu, Pr = 1.03, 0.97, 0.1, 0.71
    g = Ra * mu ** 2 / ((Th - Tl) * n ** 3 * Pr)
    return dict(nx=n, ny=n, tau_f=0.5 + 3 * mu, tau_g=0.5 + 3 * mu / Pr, G=1.0, beta=0.0, eos="ideal",
                R=1.0 / 3.0, cv=1.0, gx=0.0, gy=-g, wall_x=True, wall_y=True,
                thermal_left="dirichlet", thermal_right="dirichlet", thermal_bottom="adiabatic",
                thermal_top="adiabatic", T_left=Th, T_right=Tl, eos_fixed_T=False, T_eos=1.0)


def test_cavity_fd_and_corrected_agree_plain_departs():
    """Sec. III.B: the temperature fields of Eq. (24) and Eq. (26) nearly
    coincide, those of Eq. (7) do not (a 40^2 cavity, Ra = 10^3 by Eq. (28),
    8000 steps from rest)."""
    n = 40
    out = {}
    for tr in (PLAIN, CORRECTED, FD_RK2):
        o = Oracle(_cavity(n, 1e3))
        o.init_fields(np.ones((n, n)), np.ones((n, n)))
        assert o.step(8000, tr) == 0
        out[tr] = o.moments()[3]
    d_fd = np.abs(out[FD_RK2] - out[CORRECTED]).max()
    d_plain = np.abs(out[PLAIN] - out[CORRECTED]).max()
    print("cavity max |T - T_corrected|: fd", d_fd, "plain", d_plain)
    assert d_fd < 0.2 * d_plain, (d_fd, d_plain)


def _adiabatic_slope(nx, steps, cv, treatment=FD_RK2, phi_divu=True):
    p = dict(nx=nx, ny=4, tau_f=0.6, tau_g=0.500001, G=1.0, beta=0.0, eos="ideal", R=1.0 / 3.0, cv=cv,
             gx=0.0, gy=0.0, wall_x=False, wall_y=False, eos_fixed_T=False, T_eos=1.0, phi_divu=phi_divu)
    x = np.arange(nx)
    rho = np.tile(1.0 + 1e-3 * np.cos(2 * np.pi * x / nx), (4, 1))
    o = Oracle(p)
    o.init_fields(rho, np.ones((4, nx)))
    r0, _, _, T0 = o.moments()
    assert o.step(steps, treatment) == 0
    r1, _, _, T1 = o.moments()
    dr, dT = (r1 - r0).ravel(), (T1 - T0).ravel()
    return float(dr @ dT / (dr @ dr))


@pytest.mark.parametrize("treatment", [FD_RK2, CORRECTED, PLAIN])
@pytest.mark.parametrize("cv", [1.0, 2.0])
def test_phi_divu_gives_the_adiabatic_temperature_of_a_sound_wave(cv, treatment):
    """With the phi div u term of Eq. (5) kept, an ideal gas (p = rho R T,
    phi = -rho R T) compressed by a sound wave without conduction heats
    adiabatically: dT/T = (R/cv) drho/rho.  The slope converges to R/cv at
    first order in the acoustic scaling (t ~ n), for the finite-difference
    treatment (the term in K(T)) and for both LB treatments (the source
    w_i phi div u in the g update); without the term T hardly changes."""
    want = (1.0 / 3.0) / cv
    e1 = _adiabatic_slope(64, 20, cv, treatment) / want - 1
    e2 = _adiabatic_slope(128, 40, cv, treatment) / want - 1
    assert abs(e2) < 0.03
    assert 1.6 < e1 / e2 < 2.4, (e1, e2)
    assert abs(_adiabatic_slope(64, 20, cv, treatment, phi_divu=False)) < 1e-3 * want
