"""The natural-convection cavity of Sec. III.B against the values Table II
prints (tests/golden/table2_cavity.json), at Ra = 10^3 on 100^2.

The paper does not state its wall treatment of psi^2 or its Nusselt
estimator; with this library's walls (halfway bounce-back, mirrored psi^2
ghost) and the mean two-node temperature gradient at the hot wall, the two
forcing-term-free treatments land within 4 % of the printed 1.118 and
within 1.5 % of each other, and the plain treatment's Nusselt number is
raised well above them (the printed 4.884 depends on the unstated wall
treatment; the sign and size of the gap are what is checked)."""
import json
import os

import numpy as np
import pytest

from gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table2_cavity.json")


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _cavity(n, Ra, Th, Tl, mu, Pr):
    g = Ra * mu ** 2 / ((1.0 / (0.5 * (Th + Tl))) * (Th - Tl) * n ** 3 * Pr)
    return dict(nx=n, ny=n, tau_f=0.5 + 3 * mu, tau_g=0.5 + 3 * mu / Pr, G=1.0, beta=0.0, eos="ideal",
                R=1.0 / 3.0, cv=1.0, gx=0.0, gy=-g, wall_x=True, wall_y=True,
                thermal_left="dirichlet", thermal_right="dirichlet", thermal_bottom="adiabatic",
                thermal_top="adiabatic", T_left=Th, T_right=Tl, eos_fixed_T=False, T_eos=1.0)


def _nusselt(p, treatment, chunk, max_chunks):
    from paper_1405_2232_amd.lbm import Lattice
    n = p["nx"]
    g = Lattice(p, "fp64")
    g.init_fields(np.ones((n, n)), np.ones((n, n)))
    prev = None
    for _ in range(max_chunks):
        g.step(chunk, treatment)
        T = g.moments()[3]
        nu = float(np.mean(-(T[:, 1] - T[:, 0]) * n / (p["T_left"] - p["T_right"])))
        if prev is not None and abs(nu - prev) < 1e-6:
            break
        prev = nu
    return nu


def test_table2_cavity_ra1e3():
    from paper_1405_2232_amd.lbm import CORRECTED, FD_RK2, PLAIN
    gold = json.load(open(GOLDEN))
    s = gold["setup"]
    p = _cavity(s["n"], s["Ra"], s["Th"], s["Tl"], s["mu"], s["Pr"])
    nu_c = _nusselt(p, CORRECTED, 20000, 10)
    nu_fd = _nusselt(p, FD_RK2, 20000, 10)
    nu_p = _nusselt(p, PLAIN, 100000, 14)
    say("cavity Ra=1e3 Nu: corrected", nu_c, "finite difference", nu_fd, "plain", nu_p, "printed", gold["nu"])
    assert abs(nu_c - gold["nu"]["corrected_eq24"]) <= 0.04 * gold["nu"]["corrected_eq24"]
    assert abs(nu_fd - gold["nu"]["finite_difference_eq26"]) <= 0.04 * gold["nu"]["finite_difference_eq26"]
    assert abs(nu_c - nu_fd) <= 0.015 * nu_fd
    assert nu_p > 1.2 * nu_c
