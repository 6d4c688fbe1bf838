"""The pins have teeth: each plausible mistake below is planted in a copy of
the oracle's C source (on the CPU only), the copy is compiled and loaded in
place of the oracle, and at least one pin must then fail.  A mistake that no
pin catches would leave that part of the oracle unpinned."""
import contextlib
import os
import shutil
import subprocess
import tempfile

import pytest

import oracle.build as _build
import oracle.lbmref as _ref

import test_oracle_channel as channel
import test_oracle_fd as fd
import test_oracle_pins as pins
import test_oracle_walls as walls


def _channel_poiseuille():
    channel.test_poiseuille_flux_outlet_density_and_profile()


def _case_a_inlet():
    walls.test_inlet_holds_the_inflow_temperature(walls._steady(walls._channel(120, 20, 1.03, 0.97), 1.0, 30000))


def _case_a_outlet():
    walls.test_outlet_carries_the_channel_temperature_out(
        walls._steady(walls._channel(120, 20, 1.03, 0.97), 1.0, 30000))


def _covariance(walls_index, treatment):
    return lambda: walls.test_walled_box_is_covariant_under_exchange_of_x_and_y(walls_index, treatment)

SRC = os.path.join(os.path.dirname(_build.__file__), "lbmref.c")
HDR = os.path.join(os.path.dirname(_build.__file__), "lbmref.h")


@contextlib.contextmanager
def mutated(find, repl):
    src = open(SRC).read()
    assert src.count(find) == 1, find
    d = tempfile.mkdtemp(prefix="lbmref_mut_")
    try:
        shutil.copy(HDR, d)
        c = os.path.join(d, "lbmref.c")
        with open(c, "w") as fp:
            fp.write(src.replace(find, repl))
        so = os.path.join(d, "liblbmref_mut.so")
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-std=c11", "-shared", "-fPIC",
                               "-o", so, c, "-lm"])
        saved_lib, saved_path = _ref._lib, _build.LIB
        _ref._lib, _build.LIB = None, so
        try:
            yield
        finally:
            _ref._lib, _build.LIB = saved_lib, saved_path
    finally:
        shutil.rmtree(d, ignore_errors=True)


def _fails(fn):
    try:
        fn()
    except Exception:  # an assertion, or the run breaking down
        return True
    return False


MUTATIONS = [
    ("equilibrium drops the u^2 term's c_s^2",
     "- 0.5 * uu / CS2);", "- 0.5 * uu);",
     [lambda: pins.test_feq_moments(0)]),
    ("forcing prefactor 1 - 1/tau instead of 1 - 1/(2 tau)",
     "out[i] = (1.0 - 1.0 / (2.0 * tau_f)) * W[i] * (cx * Fx + cy * Fy);",
     "out[i] = (1.0 - 1.0 / tau_f) * W[i] * (cx * Fx + cy * Fy);",
     [lambda: pins.test_guo_forcing_moments(0)]),
    ("forcing term loses its (e.u) e part",
     "double cx = (EX[i] - ux) / CS2 + eu * EX[i] / (CS2 * CS2);",
     "double cx = (EX[i] - ux) / CS2;",
     [lambda: pins.test_guo_forcing_moments(0)]),
    ("correction term with the wrong sign",
     "out[i] = (1.0 - 1.0 / (2.0 * tau_g)) * W[i] * cvT * eF / CS2;",
     "out[i] = -(1.0 - 1.0 / (2.0 * tau_g)) * W[i] * cvT * eF / CS2;",
     [lambda: pins.test_correction_term_moments(0),
      pins.test_one_step_treatment_gap_is_divergence_of_correction_flux]),
    ("diagonal interaction weight 1/6 instead of 1/12",
     "if (e2 == 2) return 1.0 / 12.0;", "if (e2 == 2) return 1.0 / 6.0;",
     [lambda: pins.test_force_stencil_taylor_exact_for_quartics(0)]),
    ("psi^2 with + rho c_s^2",
     "double s = 2.0 * (lbmref_pressure(p, r, Te) - r * CS2) / p->G;",
     "double s = 2.0 * (lbmref_pressure(p, r, Te) + r * CS2) / p->G;",
     [lambda: pins.test_force_long_wave_limit(1.0)]),
    ("f relaxes with tau_g",
     "double fs = fi - (fi - feq[i]) / p->tau_f + fi_force[i];",
     "double fs = fi - (fi - feq[i]) / p->tau_g + fi_force[i];",
     [lambda: pins.test_shear_wave_decay_viscosity(1.0)]),
    ("g equilibrium without c_v",
     "double geq = cvT * feq[i];", "double geq = h->T[c] * feq[i];",
     [pins.test_cv_only_scales_the_energy]),
    ("mixed force with (1 - beta) instead of (1 - beta)/2",
     "Fx[c] = -G * (beta * psi[c] * s1x + 0.5 * (1.0 - beta) * s2x);",
     "Fx[c] = -G * (beta * psi[c] * s1x + (1.0 - beta) * s2x);",
     [lambda: pins.test_force_long_wave_limit(0.0)]),
    ("gravity enters with the wrong sign",
     "Fy[c] += h->rho[c] * p->gy;", "Fy[c] -= h->rho[c] * p->gy;",
     [pins.test_momentum_budget_with_gravity]),
    ("adiabatic wall anti-bounces back",
     "r * Tw;\n          else\n            h->g2[PL(h, o) + c] = gs;",
     "r * Tw;\n          else\n            h->g2[PL(h, o) + c] = -gs;",
     [pins.test_adiabatic_walls_conserve_energy]),
    ("Carnahan-Starling numerator with + eta^3",
     "double num = 1.0 + eta + eta * eta - eta * eta * eta;\n  double den = (1.0 - eta) * (1.0 - eta) * (1.0 - eta);\n  return rho * p->R * T",
     "double num = 1.0 + eta + eta * eta + eta * eta * eta;\n  double den = (1.0 - eta) * (1.0 - eta) * (1.0 - eta);\n  return rho * p->R * T",
     [pins.test_cs_eos_critical_point]),
    ("velocity without the half force",
     "      double ux = (h->jx[c] + 0.5 * Fx[c]) / r;\n      double uy = (h->jy[c] + 0.5 * Fy[c]) / r;\n      if (!src) {",
     "      double ux = h->jx[c] / r;\n      double uy = h->jy[c] / r;\n      if (!src) {",
     [pins.test_momentum_budget_with_gravity, lambda: pins.test_slab_steady_state_forcing_term_effect(1.0)]),
    ("temperature moment without c_v",
     "h->T[c] = e / (r * p->cv);", "h->T[c] = e / r;",
     [pins.test_cv_only_scales_the_energy]),
    ("Dirichlet wall bounces back instead of anti-bouncing",
     "h->g2[PL(h, o) + c] = -gs + 2.0 * W[i] * p->cv * r * Tw;",
     "h->g2[PL(h, o) + c] = gs + 2.0 * W[i] * p->cv * r * Tw;",
     [lambda: pins.test_linear_conduction_between_dirichlet_walls(0.8)]),
    ("psi ghost beyond a wall wraps periodically",
     "if (y < 0) y = wall_y ? 0 : y + ny;", "if (y < 0) y = y + ny;",
     [pins.test_force_wall_mirror_ghost]),
    ("streaming pushes the wrong way",
     "int xn = x + EX[i], yn = y + EY[i];", "int xn = x - EX[i], yn = y - EY[i];",
     [pins.test_density_wave_is_carried_by_a_uniform_flow]),
    ("second Runge-Kutta stage at half the step (the printed form)",
     "h->Ts[c] = h->T[c] + h->K1[c];", "h->Ts[c] = h->T[c] + 0.5 * h->K1[c];",
     [fd.test_one_step_matches_independent_numpy, fd.test_gaussian_diffusion_second_order]),
    ("finite-difference Laplacian without the factor 2",
     "lapT += 2.0 * w * (Tn - T[c]);", "lapT += w * (Tn - T[c]);",
     [fd.test_one_step_matches_independent_numpy]),
    ("inlet bounce-back without the inlet momentum",
     "h->f2[PL(h, o) + c] = fs - 2.0 * W[i] * r * eu / CS2;", "h->f2[PL(h, o) + c] = fs;",
     [_channel_poiseuille]),
    ("outlet anti-bounce-back with the wrong sign",
     "h->f2[PL(h, o) + c] = -fs + 2.0 * W[i] * p->rho_out * even;",
     "h->f2[PL(h, o) + c] = fs + 2.0 * W[i] * p->rho_out * even;",
     [_channel_poiseuille]),
    ("phi div u with the wrong sign",
     "  return phi * du;\n}", "  return -phi * du;\n}",
     [lambda: fd.test_phi_divu_gives_the_adiabatic_temperature_of_a_sound_wave(1.0, 2)]),
    ("LB source phi div u without its weights",
     "if (src) gs += W[i] * S;", "if (src) gs += S;",
     [lambda: fd.test_phi_divu_gives_the_adiabatic_temperature_of_a_sound_wave(1.0, 1)]),
    ("LB source phi div u left out of the plain treatment",
     "const int src = p->phi_divu && treatment != LBMREF_FD_RK2;",
     "const int src = p->phi_divu && treatment == LBMREF_CORRECTED;",
     [lambda: fd.test_phi_divu_gives_the_adiabatic_temperature_of_a_sound_wave(1.0, 0)]),
    ("finite-difference Dirichlet ghost equal to the wall value",
     "int th = wall_condition(p, sx, sy, &Tw);\n  return th == LBMREF_THERMAL_DIRICHLET ? 2.0 * Tw - v : v;",
     "int th = wall_condition(p, sx, sy, &Tw);\n  return th == LBMREF_THERMAL_DIRICHLET ? Tw : v;",
     [lambda: fd.test_linear_conduction_is_a_fixed_point_and_the_limit(0.6)]),
    ("inlet g equilibrium without its velocity terms",
     "(1.0 + 4.5 * eu * eu - 1.5 * p->u_in * p->u_in);", "1.0;",
     [_case_a_inlet]),
    ("inlet g bounces back",
     "h->g2[PL(h, o) + c] = -gs + 2.0 * W[i] * p->cv * r * p->T_left *",
     "h->g2[PL(h, o) + c] = gs + 0.0 * W[i] * p->cv * r * p->T_left *",
     [lambda: walls.test_isothermal_channel_stays_at_its_temperature(1)]),
    ("outlet g holds the inflow temperature",
     "h->g2[PL(h, o) + c] = -gs + 2.0 * W[i] * cvT * r * even;",
     "h->g2[PL(h, o) + c] = -gs + 2.0 * W[i] * p->cv * p->T_left * r * even;",
     [_case_a_outlet]),
    ("outlet g bounces back",
     "h->g2[PL(h, o) + c] = -gs + 2.0 * W[i] * cvT * r * even;",
     "h->g2[PL(h, o) + c] = gs;",
     [walls.test_adiabatic_channel_fills_with_the_inflow_temperature]),
    ("outlet g equilibrium without its velocity terms",
     "h->g2[PL(h, o) + c] = -gs + 2.0 * W[i] * cvT * r * even;",
     "h->g2[PL(h, o) + c] = -gs + 2.0 * W[i] * cvT * r;",
     [lambda: walls.test_isothermal_channel_stays_at_its_temperature(1)]),
    ("the y wall wins at box corners",
     "int sx = hit_x && !open ? (xn < 0 ? 0 : 1) : -1;",
     "int sx = hit_x && !open && !hit_y ? (xn < 0 ? 0 : 1) : -1;",
     [_covariance(1, 1), _covariance(2, 1)]),
    ("a Dirichlet corner takes one wall's temperature",
     "*Tw = 0.5 * (tw[sx] + tw[sy]);", "*Tw = tw[sy];",
     [_covariance(0, 1)]),
    ("finite-difference ghost: the y wall wins at box corners",
     "if (p->wall_x == 2 && sy >= 0) sx = -1;", "if (sy >= 0) sx = -1;",
     [_covariance(0, 2), _covariance(2, 2)]),
]


@pytest.mark.parametrize("name,find,repl,checks", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(name, find, repl, checks):
    with mutated(find, repl):
        caught = [_fails(fn) for fn in checks]
    assert any(caught), "no pin catches: " + name


def test_unmutated_copy_passes_the_same_checks():
    """Control: the copy mechanism itself breaks nothing."""
    with mutated("static const double CS2 = 1.0 / 3.0;", "static const double CS2 = 1.0 / 3.0;"):
        for _, _, _, checks in MUTATIONS[:6]:
            for fn in checks:
                assert not _fails(fn)
