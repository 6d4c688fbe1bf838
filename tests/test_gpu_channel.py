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


def _nusselt_fully_developed(p, treatment, steps):
    """Nu(x) = D_h q_w / (lambda (T_w - T_b)) at the top wall, D_h = 2 H,
    the wall gradient from the two nodes next to the wall, T_b the
    mass-flux-weighted bulk temperature; averaged over the third quarter of
    the channel (thermally developed, away from the outlet's influence)."""
    from paper_1405_2232_amd.lbm import Lattice
    nx, ny = p["nx"], p["ny"]
    g = Lattice(p, "fp64")
    g.init_fields(np.ones((ny, nx)), np.ones((ny, nx)))
    g.step(steps, treatment)
    r, ux, uy, T = g.moments()
    Tw = p["T_top"]
    Tb = (r * ux * T).sum(0) / (r * ux).sum(0)
    nu = 2 * ny * (T[-1] - T[-2]) / (Tw - Tb)
    return float(np.mean(nu[nx // 2: 3 * nx // 4]))


def test_table1_fully_developed_nusselt():
    gold = json.load(open(GOLDEN))
    out = {}
    for case in ("A", "B"):
        p = channel(500, 60, case)
        for tr in (FD_RK2, CORRECTED):
            out[(case, tr)] = _nusselt_fully_developed(p, tr, 150000)
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
