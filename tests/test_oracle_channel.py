"""Pins of the oracle's open channel (inlet/outlet of Sec. III.A, a
reading: the paper states uniform inflow and fully developed outflow only).

- Single phase, isothermal: mass flux is the same through every cross
  section at steady state, the outlet holds its density, and the developed
  profile is the Poiseuille parabola between halfway walls.
- The finite-difference temperature treatment (Eqs. (26)-(27)) reaches the
  analytic fully developed Nusselt number 7.54 of Case A (both plates at
  T_w), the value Table I compares with.
"""
import numpy as np

from oracle import CORRECTED, FD_RK2, Oracle


def _channel(nx, ny, case="A", G=1.0, u_in=0.05):
    mu, Pr = 0.1, 0.71
    return dict(nx=nx, ny=ny, tau_f=0.5 + 3 * mu, tau_g=0.5 + 3 * mu / Pr, G=G, beta=0.0, eos="ideal",
                R=1.0 / 3.0, cv=1.0, gx=0.0, gy=0.0, wall_x="open", wall_y=True,
                thermal_left="dirichlet", thermal_right="adiabatic",
                thermal_bottom="dirichlet" if case == "A" else "adiabatic", thermal_top="dirichlet",
                T_left=1.03, T_bottom=0.97, T_top=0.97, u_in=u_in, rho_out=1.0, eos_fixed_T=False, T_eos=1.0)


def test_poiseuille_flux_outlet_density_and_profile():
    nx, ny = 160, 16
    p = _channel(nx, ny, G=0.0)
    p.update(T_left=1.0, T_bottom=1.0, T_top=1.0)
    o = Oracle(p)
    o.init_fields(np.ones((ny, nx)), np.ones((ny, nx)))
    assert o.step(30000, CORRECTED) == 0
    r, ux, uy, T = o.moments()
    flux = (r * ux).sum(0)
    assert np.abs(flux[2:-2] - flux[nx // 2]).max() < 1e-9 * flux[nx // 2]
    assert abs(r[:, -1].mean() - 1.0) < 2e-3
    y = np.arange(ny) + 0.5
    shape = 1.0 - (2.0 * y / ny - 1.0) ** 2
    prof = ux[:, 3 * nx // 4]
    fit = prof @ shape / (shape @ shape)
    assert np.abs(prof - fit * shape).max() < 2e-3 * prof.max()
    assert np.abs(uy[:, 3 * nx // 4]).max() < 1e-6


def test_fd_case_a_fully_developed_nusselt():
    nx, ny = 240, 30
    p = _channel(nx, ny, "A")
    o = Oracle(p)
    o.init_fields(np.ones((ny, nx)), np.ones((ny, nx)))
    assert o.step(40000, FD_RK2) == 0
    r, ux, uy, T = o.moments()
    Tb = (r * ux * T).sum(0) / (r * ux).sum(0)
    nu = 2 * ny * (T[-1] - T[-2]) / (0.97 - Tb)
    nu_dev = float(np.mean(nu[nx // 2: 3 * nx // 4]))
    print("FD case A developed Nu", nu_dev)
    assert abs(nu_dev - 7.54) < 0.02 * 7.54
