"""Seeded synthetic inputs for the thermal pseudopotential LB workloads.

This module builds initial fields (density, temperature) and parameter
dicts; it holds none of the LB step's arithmetic.  Both the HIP path and
the CPU oracle take their inputs from here, so neither side generates
random numbers of its own.

Two-phase initial states sit between the coexistence densities of the
Carnahan-Starling (CS) equation of state, found by Maxwell's equal-area
construction at the initial temperature.  The CS constants a = 1, b = 4,
R = 1 give T_c = 0.3773 a / (b R).  (The paper's own benchmarks use the
ideal EOS; the CS two-phase states are the workloads of this library.)
All randomness comes from numpy's PCG64 with a stated seed.
"""
import math

import numpy as np
from scipy.optimize import brentq

CS_A, CS_B, CS_R = 1.0, 4.0, 1.0


def cs_tc(a=CS_A, b=CS_B, R=CS_R):
    """Critical temperature of the CS EOS, 0.3773 a/(b R)."""
    return 0.3773 * a / (b * R)


# --- CS EOS for the initial-condition construction only ---------------------

def _cs_p(rho, T, a, b, R):
    eta = b * rho / 4.0
    return rho * R * T * (1 + eta + eta ** 2 - eta ** 3) / (1 - eta) ** 3 - a * rho ** 2


def _cs_dpdrho(rho, T, a, b, R, h=1e-7):
    return (_cs_p(rho + h, T, a, b, R) - _cs_p(rho - h, T, a, b, R)) / (2 * h)


def _cs_mu(rho, T, a, b, R):
    """Chemical potential (up to a T-dependent constant): the CS excess part
    (8 eta - 9 eta^2 + 3 eta^3)/(1 - eta)^3 plus the ideal log and -2 a rho."""
    eta = b * rho / 4.0
    return R * T * (math.log(rho) + (8 * eta - 9 * eta ** 2 + 3 * eta ** 3) / (1 - eta) ** 3) - 2 * a * rho


def maxwell_densities(T, a=CS_A, b=CS_B, R=CS_R):
    """Coexistence densities (rho_v, rho_l) of the CS EOS at T < T_c by the
    equal-area (equal chemical potential and pressure) construction."""
    if not T < cs_tc(a, b, R):
        raise ValueError("T must be below the critical temperature")
    rmax = 4.0 / b
    grid = np.linspace(1e-6, rmax * 0.95, 20001)
    d = np.array([_cs_dpdrho(r, T, a, b, R) for r in grid])
    sc = np.where(np.sign(d[:-1]) != np.sign(d[1:]))[0]
    if len(sc) < 2:
        raise ValueError("no van der Waals loop at this temperature")
    s1 = brentq(lambda r: _cs_dpdrho(r, T, a, b, R), grid[sc[0]], grid[sc[0] + 1], xtol=1e-15)
    s2 = brentq(lambda r: _cs_dpdrho(r, T, a, b, R), grid[sc[1]], grid[sc[1] + 1], xtol=1e-15)
    p_hi = _cs_p(s1, T, a, b, R)
    p_lo = max(_cs_p(s2, T, a, b, R), 1e-14)

    def roots(P):
        rv = brentq(lambda r: _cs_p(r, T, a, b, R) - P, 1e-14, s1, xtol=1e-16, rtol=1e-15)
        rl = brentq(lambda r: _cs_p(r, T, a, b, R) - P, s2, rmax * 0.999, xtol=1e-16, rtol=1e-15)
        return rv, rl

    def dmu(P):
        rv, rl = roots(P)
        return _cs_mu(rl, T, a, b, R) - _cs_mu(rv, T, a, b, R)

    eps = 1e-12 * (p_hi - p_lo)
    P = brentq(dmu, p_lo + eps, p_hi - eps, xtol=1e-18, rtol=1e-15)
    return roots(P)


# --- profiles ----------------------------------------------------------------

def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def tanh_step(d, W=2.0):
    """Smooth indicator: 1 well inside (d << 0), 0 well outside (d >> 0)."""
    return 0.5 * (1.0 - np.tanh(2.0 * d / W))


def droplet_field(nx, ny, rho_v, rho_l, R, cx=None, cy=None, W=2.0):
    """Single circular droplet of radius R centred at node (cx, cy)."""
    cx = nx / 2 if cx is None else cx
    cy = ny / 2 if cy is None else cy
    x = np.arange(nx)[None, :]
    y = np.arange(ny)[:, None]
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
    return rho_v + (rho_l - rho_v) * tanh_step(r - R, W)


def slab_field(nx, ny, rho_v, rho_l, W=2.0):
    """Flat liquid slab between y = ny/4 and y = 3 ny/4, vapour elsewhere."""
    y = np.arange(ny, dtype=np.float64)[:, None]
    prof = rho_v + 0.5 * (rho_l - rho_v) * (np.tanh(2 * (y - ny / 4) / W) - np.tanh(2 * (y - 3 * ny / 4) / W))
    return np.broadcast_to(prof, (ny, nx)).copy()


def multi_droplet_field(nx, ny, rho_v, rho_l, centres, radii, W=2.0, periodic_x=True, periodic_y=False):
    """Non-overlapping droplets: rho_v + (rho_l - rho_v) * max_k indicator_k."""
    chi = np.zeros((ny, nx))
    for (cx, cy), R in zip(centres, radii):
        m = int(math.ceil(R + 4 * W)) + 1
        xs = np.arange(int(math.floor(cx)) - m, int(math.ceil(cx)) + m + 1)
        ys = np.arange(int(math.floor(cy)) - m, int(math.ceil(cy)) + m + 1)
        if periodic_x:
            xi = np.mod(xs, nx)
        else:
            keep = (xs >= 0) & (xs < nx)
            xs, xi = xs[keep], xs[keep]
        if periodic_y:
            yi = np.mod(ys, ny)
        else:
            keep = (ys >= 0) & (ys < ny)
            ys, yi = ys[keep], ys[keep]
        r = np.sqrt((xs[None, :] - cx) ** 2 + (ys[:, None] - cy) ** 2)
        sub = tanh_step(r - R, W)
        blk = chi[np.ix_(yi, xi)]
        chi[np.ix_(yi, xi)] = np.maximum(blk, sub)
    return rho_v + (rho_l - rho_v) * chi


def place_droplets(rng, nx, ny, n, rmin, rmax, gap=4.0, wall_margin=4.0, periodic_x=True,
                   max_tries=200000):
    """Random non-overlapping circles (periodic in x, walls in y)."""
    centres, radii = [], []
    tries = 0
    while len(radii) < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place %d droplets" % n)
        R = rng.uniform(rmin, rmax)
        cx = rng.uniform(0, nx)
        cy = rng.uniform(R + wall_margin, ny - R - wall_margin)
        ok = True
        for (px, py), pr in zip(centres, radii):
            dx = abs(cx - px)
            if periodic_x:
                dx = min(dx, nx - dx)
            if math.hypot(dx, cy - py) < R + pr + gap:
                ok = False
                break
        if ok:
            centres.append((cx, cy))
            radii.append(R)
    return centres, radii


def noise(rng, field, rel):
    """Multiplicative uniform noise field * (1 + rel U[-1, 1])."""
    return field * (1.0 + rel * rng.uniform(-1.0, 1.0, size=field.shape))


# --- workloads -----------------------------------------------------------------

def base_params(nx, ny, T0, tau_f=1.0, tau_g=0.8):
    return dict(nx=nx, ny=ny, tau_f=tau_f, tau_g=tau_g, G=-1.0, beta=1.0, eos="cs",
                a=CS_A, b=CS_B, R=CS_R, cv=1.0, gx=0.0, gy=0.0, wall_x=False, wall_y=False,
                eos_fixed_T=False, T_eos=T0)


def static_droplet(nx=64, ny=64, radius=16.0, T_ratio=0.85, tau_f=1.0, tau_g=0.8, seed=0,
                   rho_noise=0.01, T_noise=0.005):
    """Periodic static droplet: radius-16 tanh droplet (width 2) between the
    Maxwell densities at T0 = 0.85 T_c, +-1% density and +-0.5% temperature
    noise (the 64x64 two-treatment parity workload)."""
    Tc = cs_tc()
    T0 = T_ratio * Tc
    rv, rl = maxwell_densities(T0)
    rng = _rng(seed)
    rho = droplet_field(nx, ny, rv, rl, radius)
    rho = noise(rng, rho, rho_noise)
    T = noise(rng, np.full((ny, nx), T0), T_noise)
    p = base_params(nx, ny, T0, tau_f, tau_g)
    return p, rho, T


def wall_slab(nx=2048, ny=2048, T_ratio=0.85, T_bottom_ratio=0.80, T_top_ratio=0.90):
    """Flat liquid slab in the middle half, periodic in x, walls in y with
    Dirichlet temperatures 0.80 T_c (bottom) and 0.90 T_c (top); uniform
    initial T = 0.85 T_c, no noise (the 2048x2048 throughput workload)."""
    Tc = cs_tc()
    T0 = T_ratio * Tc
    rv, rl = maxwell_densities(T0)
    rho = slab_field(nx, ny, rv, rl)
    T = np.full((ny, nx), T0)
    p = base_params(nx, ny, T0)
    p.update(wall_y=True, thermal_bottom="dirichlet", thermal_top="dirichlet",
             T_bottom=T_bottom_ratio * Tc, T_top=T_top_ratio * Tc)
    return p, rho, T


_SIDES = np.arange(64, 513, 32)


# Stable range of the static droplet with these EOS constants, Guo forcing
# and the EOS at the local temperature, measured over 20,000 steps on
# 128^2..480x128 lattices: at 0.80 T_c every case diverges; at 0.84 T_c
# tau_f < 0.7 diverges within 1,000-8,000 steps; tau_g = 1.2 destabilises
# even 0.86 T_c within 6,000-18,000 steps, tau_g = 0.6 does not.
STABLE_T_RATIO = (0.86, 0.95)
STABLE_TAU_F = (0.7, 1.2)
STABLE_TAU_G = (0.6, 0.9)


def batch_lattices(count=256, seed=2, t_ratio=STABLE_T_RATIO, tau_f_range=STABLE_TAU_F,
                   tau_g_range=STABLE_TAU_G):
    """Uneven batch of periodic static droplets: sides uniform in
    {64, 96, ..., 512}, radius U[0.15, 0.35] min side, T0/T_c, tau_f and
    tau_g uniform in the model's stable range (0.86-0.95, 0.7-1.2,
    0.6-0.9); +-1% / +-0.5% noise."""
    rng = _rng(seed)
    Tc = cs_tc()
    out = []
    for _ in range(count):
        nx = int(rng.choice(_SIDES))
        ny = int(rng.choice(_SIDES))
        R = rng.uniform(0.15, 0.35) * min(nx, ny)
        tr = rng.uniform(*t_ratio)
        tau_f = rng.uniform(*tau_f_range)
        tau_g = rng.uniform(*tau_g_range)
        T0 = tr * Tc
        rv, rl = maxwell_densities(T0)
        rho = noise(rng, droplet_field(nx, ny, rv, rl, R), 0.01)
        T = noise(rng, np.full((ny, nx), T0), 0.005)
        out.append((base_params(nx, ny, T0, tau_f, tau_g), rho, T))
    return out


def warmstart_case(seed, n=128, rmin=8.0, rmax=48.0, max_drops=6, t_ratio=(0.86, 0.92),
                   dT_ratio=(0.0, 0.04), tau_f_range=(0.8, 1.2), tau_g_range=STABLE_TAU_G):
    """Steady-state case of the warm start: 1-6 droplets of radius 8-48
    (at most n/(4 sqrt(k)) for k droplets) in an n x n box, periodic in x, Dirichlet walls in y
    holding a linear temperature difference dT, initial T the conduction
    profile; T0/T_c in [0.86, 0.92], dT/T_c in [0, 0.04], tau_f in
    [0.8, 1.2], tau_g in [0.6, 0.9].  The EOS is evaluated at T0 (with the
    EOS at the local temperature these states have no steady state)."""
    rng = _rng(seed)
    Tc = cs_tc()
    tr = rng.uniform(*t_ratio)
    dT = rng.uniform(*dT_ratio) * Tc
    T0 = tr * Tc
    tau_f = rng.uniform(*tau_f_range)
    tau_g = rng.uniform(*tau_g_range)
    k = int(rng.integers(1, max_drops + 1))
    rv, rl = maxwell_densities(T0)
    rmax_eff = max(rmin, min(rmax, 0.25 * n / math.sqrt(k)))
    centres, radii = place_droplets(rng, n, n, k, rmin, rmax_eff)
    rho = multi_droplet_field(n, n, rv, rl, centres, radii)
    y = (np.arange(n) + 0.5) / n
    Tb, Tt = T0 - 0.5 * dT, T0 + 0.5 * dT
    T = np.broadcast_to((Tb + (Tt - Tb) * y)[:, None], (n, n)).copy()
    p = base_params(n, n, T0, tau_f, tau_g)
    p.update(wall_y=True, thermal_bottom="dirichlet", thermal_top="dirichlet", T_bottom=Tb, T_top=Tt,
             eos_fixed_T=True)
    return p, rho, T


def many_droplets_gravity(nx=4096, ny=4096, count=200, seed=4, rmin=8.0, rmax=40.0, g=1e-6,
                          T_bottom_ratio=0.86, T_top_ratio=0.94):
    """Large two-phase case: 200 non-overlapping droplets (radius 8-40),
    gravity 1e-6 in -y, walls at 0.86 T_c (bottom) and 0.94 T_c (top) (a
    colder wall, e.g. 0.75 T_c, takes the droplets beside it out of the
    model's stable range and the run diverges within 2000 steps), initial T
    the linear conduction profile, densities from Maxwell at the wall mean."""
    rng = _rng(seed)
    Tc = cs_tc()
    Tb, Tt = T_bottom_ratio * Tc, T_top_ratio * Tc
    Tm = 0.5 * (Tb + Tt)
    rv, rl = maxwell_densities(Tm)
    centres, radii = place_droplets(rng, nx, ny, count, rmin, rmax)
    rho = multi_droplet_field(nx, ny, rv, rl, centres, radii)
    y = (np.arange(ny) + 0.5) / ny
    T = np.broadcast_to((Tb + (Tt - Tb) * y)[:, None], (ny, nx)).copy()
    p = base_params(nx, ny, Tm)
    p.update(wall_y=True, thermal_bottom="dirichlet", thermal_top="dirichlet", T_bottom=Tb,
             T_top=Tt, gy=-g)
    return p, rho, T
