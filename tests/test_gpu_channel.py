"""The open channel of Sec. III.A (uniform inflow, fully developed outflow,
walls at T_w): GPU parity with the oracle for the three temperature
treatments, and the fully developed Nusselt numbers against Table I
(tests/golden/table1_channel.json)."""
import json
import os

import numpy as np
import pytest

from gpu_util import compare_fp32dev, compare_fp64, gpu_run, need_gpu, oracle_run, say
from oracle import CORRECTED, FD_RK2, PLAIN

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table1_channel.json")


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def channel(nx, ny, case, u_in=0.05, Tin=1.03, Tw=0.97, mu=0.1, Pr=0.71):
    return dict(nx=nx, ny=ny, tau_f=0.5 + 3 * mu, tau_g=0.5 + 3 * mu / Pr, G=1.0, beta=0.0, eos="ideal",
                R=1.0 / 3.0, cv=1.0, gx=0.0, gy=0.0, wall_x="open", wall_y=True,
                thermal_left="dirichlet", thermal_right="adiabatic",
                thermal_bottom="dirichlet" if case == "A" else "adiabatic", thermal_top="dirichlet",
                T_left=Tin, T_bottom=Tw, T_top=Tw, u_in=u_in, rho_out=1.0, eos_fixed_T=False, T_eos=1.0)


@pytest.mark.parametrize("treatment", [PLAIN, CORRECTED, FD_RK2])
@pytest.mark.parametrize("precision", ["fp64", "fp32local"])
def test_channel_parity(treatment, precision):
    nx, ny = 97, 23
    p = channel(nx, ny, "B")
    one = np.ones((ny, nx))
    say("case channel", treatment, precision)
    g = gpu_run(p, one, one, 1500, treatment, precision=precision)
    o = oracle_run(p, one, one, 1500, treatment)
    if precision == "fp64":
        compare_fp64(g.moments(), o.moments(), what=("channel", treatment))
    else:
        compare_fp32dev(g.moments(), o.moments(), what=("channel fp32local", treatment))


def _nusselt_profile(p, treatment, steps):
    """Nu(x) = D_h q_w / (lambda (T_w - T_b)) at the top wall, D_h = 2 H,
    the wall gradient from the two nodes next to the wall, T_b the
    mass-flux-weighted bulk temperature.  (The quadratic through T_w half a
    spacing beyond the last node, (8 T_w - 9 T_0 + T_1)/3, suits the
    finite-difference treatment, whose ghost node holds T_w exactly halfway,
    but not the LB treatments: BGK's anti-bounce-back holds T_w at a
    distance that depends on tau_g, and for the corrected treatment that
    estimator reads 2.58 where the two-node gradient reads 7.63.)"""
    from paper_1405_2232_amd.lbm import Lattice
    nx, ny = p["nx"], p["ny"]
    g = Lattice(p, "fp64")
    g.init_fields(np.ones((ny, nx)), np.ones((ny, nx)))
    g.step(steps, treatment)
    r, ux, uy, T = g.moments()
    Tw = p["T_top"]
    Tb = (r * ux * T).sum(0) / (r * ux).sum(0)
    return 2 * ny * (T[-1] - T[-2]) / (Tw - Tb)


_PROFILES = {}


def _profile(case, treatment):
    """Nu(x) of the 500 x 60 channel after 150,000 steps (steady: the
    profiles do not change between 150,000 and 300,000 steps)."""
    key = (case, treatment)
    if key not in _PROFILES:
        _PROFILES[key] = _nusselt_profile(channel(500, 60, case), treatment, 150000)
    return _PROFILES[key]


def test_table1_fully_developed_nusselt():
    """Averaged over the third quarter of the channel (thermally developed,
    away from the outlet's influence)."""
    gold = json.load(open(GOLDEN))
    out = {(case, tr): float(np.mean(_profile(case, tr)[250:375]))
           for case in ("A", "B") for tr in (FD_RK2, CORRECTED)}
    say("channel Nu: FD A/B", out[("A", FD_RK2)], out[("B", FD_RK2)], "corrected A/B",
        out[("A", CORRECTED)], out[("B", CORRECTED)], "printed", gold["nu"])
    # the paper's own values sit 0.4 % (A) and 1 % (B) from the analytic
    # ones; these are held to 2.5 % of the printed values and 2 % of the
    # analytic ones
    for case in ("A", "B"):
        for tr, key in ((FD_RK2, "finite_difference_eq26"), (CORRECTED, "corrected_eq24")):
            printed = gold["nu"][key][case]
            assert abs(out[(case, tr)] - printed) <= 0.025 * printed, (case, tr)
        assert abs(out[(case, FD_RK2)] - gold["nu"]["analytic"][case]) <= 0.02 * gold["nu"]["analytic"][case]


def test_plain_treatment_departs_along_the_channel():
    """Nu(x) of the three treatments (Sec. III.A, Fig. 1), reported at a
    few stations.  The paper finds the plain treatment's values far from the
    other two (about 13 and 12.5 near the outlet); here it departs from them
    along the whole developed region by far more than they differ, but
    below them (3.0 and 2.9 against 7.5 and 4.8): beside the wall the
    force's y component balances the temperature gradient in the plain
    scheme's heat flux (lambda_eff,y of Eq. 23 near zero), and the printed
    values depend on wall and outlet treatments the paper does not give."""
    gold = json.load(open(GOLDEN))
    stations = [25, 50, 100, 200, 300, 400, 450, 480, 490]
    for case in ("A", "B"):
        prof = {tr: _profile(case, tr) for tr in (FD_RK2, CORRECTED, PLAIN)}
        for tr, name in ((FD_RK2, "finite difference"), (CORRECTED, "corrected"), (PLAIN, "plain")):
            say("channel", case, name, "Nu(x) at", stations, [round(float(prof[tr][x]), 3) for x in stations])
        say("printed near the outlet, plain:", gold["plain_eq7_near_outlet"][case])
        dev = slice(250, 375)
        nf, nc, npl = (float(np.mean(prof[tr][dev])) for tr in (FD_RK2, CORRECTED, PLAIN))
        spread = abs(nc - nf)
        assert abs(npl - nf) > 10 * spread + 0.1 * nf, (case, npl, nc, nf)
        # the departure holds at every station of the developed region
        for x in range(100, 450, 25):
            assert abs(prof[PLAIN][x] - prof[FD_RK2][x]) > 0.2 * prof[FD_RK2][x], (case, x)
