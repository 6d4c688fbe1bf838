"""Pins of the oracle's equilibrium start at a given fluid velocity
(init_fields_physical): with the forcing of Eq. (1) (Sec. II) the velocity
is (j + F/2)/rho, so the start stores j = rho u - F/2.  Checked against the
defining property through the oracle's moments, against a direct sum of the
stored distributions, against the plain start when no force acts, against
the zero net pseudopotential force of a periodic domain, and against the
steady state of a flat interface, where the stored momentum is -F/2."""
import numpy as np
import pytest

from oracle import CORRECTED, Oracle
from paper_1405_2232_amd import inputs

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)


def _droplet_with_flow(gravity, walls):
    p, rho, T = inputs.static_droplet(nx=40, ny=36, radius=9)
    if gravity:
        p["gx"], p["gy"] = 1e-5, -2e-5
    if walls:
        p.update(wall_y=True, thermal_bottom="dirichlet", thermal_top="dirichlet",
                 T_bottom=float(T.mean()), T_top=float(T.mean()))
    rng = np.random.default_rng(3)
    ux = rng.uniform(-0.02, 0.02, rho.shape)
    uy = rng.uniform(-0.02, 0.02, rho.shape)
    return p, rho, T, ux, uy


@pytest.mark.parametrize("gravity,walls", [(False, False), (True, False), (True, True)])
def test_reported_velocity_is_the_given_one(gravity, walls):
    p, rho, T, ux, uy = _droplet_with_flow(gravity, walls)
    o = Oracle(p)
    o.init_fields(rho, T, ux, uy)
    _, u0, _, _ = o.moments()
    Fx, Fy = o.force()
    assert np.abs(Fx).max() > 1e-3  # the interface force is not negligible
    # the plain start is off by F/(2 rho)
    assert np.abs(u0 - ux).max() > 1e-3
    o.init_fields_physical(rho, T, ux, uy)
    r, u, v, t = o.moments()
    assert np.allclose(r, rho, rtol=1e-15, atol=0)
    assert np.allclose(t, T, rtol=1e-14, atol=0)
    assert np.abs(u - ux).max() < 1e-15
    assert np.abs(v - uy).max() < 1e-15


def test_stored_momentum_is_rho_u_minus_half_force():
    p, rho, T, ux, uy = _droplet_with_flow(True, False)
    o = Oracle(p)
    o.init_fields_physical(rho, T, ux, uy)
    f, g = o.get_state()
    jx = (f * EX[:, None, None]).sum(axis=0)
    jy = (f * EY[:, None, None]).sum(axis=0)
    Fx, Fy = o.force()
    assert np.abs(jx - (rho * ux - 0.5 * Fx)).max() < 1e-15
    assert np.abs(jy - (rho * uy - 0.5 * Fy)).max() < 1e-15
    # g is cv T f (the equilibrium of Eq. (7) at the same velocity)
    assert np.allclose(g, p.get("cv", 1.0) * T[None] * f, rtol=1e-15, atol=0)


def test_without_force_equals_plain_start():
    n = 12
    rng = np.random.default_rng(6)
    p = inputs.base_params(n, n, 0.08)
    p["G"] = 0.0
    rho = rng.uniform(0.5, 1.5, (n, n))
    T = rng.uniform(0.5, 1.5, (n, n))
    ux = rng.uniform(-0.05, 0.05, (n, n))
    a, b = Oracle(p), Oracle(p)
    a.init_fields(rho, T, ux, None)
    b.init_fields_physical(rho, T, ux, None)
    fa, ga = a.get_state()
    fb, gb = b.get_state()
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)


def test_total_momentum_unchanged_on_a_periodic_lattice():
    """The pseudopotential force sums to zero over a periodic domain, so
    the physical start moves no net momentum."""
    p, rho, T, ux, uy = _droplet_with_flow(False, False)
    a, b = Oracle(p), Oracle(p)
    a.init_fields(rho, T, ux, uy)
    b.init_fields_physical(rho, T, ux, uy)
    fa, _ = a.get_state()
    fb, _ = b.get_state()
    for e in (EX, EY):
        ja = (fa * e[:, None, None]).sum()
        jb = (fb * e[:, None, None]).sum()
        assert abs(ja - jb) < 1e-13 * np.abs(fa).sum()
    assert not np.array_equal(fa, fb)


def _flat_interface():
    Tc = inputs.cs_tc()
    T0 = 0.85 * Tc
    rv, rl = inputs.maxwell_densities(T0)
    p = inputs.base_params(4, 64, T0)
    p["eos_fixed_T"] = True
    rho = inputs.slab_field(4, 64, rv, rl)
    return p, rho, np.full((64, 4), T0)


def _one_step_residual(o):
    r0, _, _, t0 = o.moments()
    o.step(1, CORRECTED)
    r1, _, _, t1 = o.moments()
    return max(np.abs(r1 - r0).max() / np.abs(r1).max(), np.abs(t1 - t0).max() / np.abs(t1).max())


def test_flat_interface_steady_state_holds_minus_half_force():
    """At the steady state of a flat interface the fluid is at rest and the
    stored momentum is -F/2; restarting from its density and temperature,
    the physical start is much closer to it than the plain start."""
    p, rho, T = _flat_interface()
    o = Oracle(p)
    o.init_fields(rho, T)
    o.step(12000, CORRECTED)
    assert _one_step_residual(o) < 1e-12
    r, u, v, t = o.moments()
    f, _ = o.get_state()
    Fx, Fy = o.force()
    jy = (f * EY[:, None, None]).sum(axis=0)
    assert np.abs(Fy).max() > 1e-3
    assert np.abs(v).max() < 1e-10  # at rest ...
    assert np.abs(jy + 0.5 * Fy).max() < 1e-10  # ... with j = -F/2
    plain, phys = Oracle(p), Oracle(p)
    plain.init_fields(r, t)
    phys.init_fields_physical(r, t)
    rp, rq = _one_step_residual(plain), _one_step_residual(phys)
    assert rq < rp / 10, (rp, rq)
