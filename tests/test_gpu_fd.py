"""GPU parity of the finite-difference temperature treatment (Eqs. (26)-(27))
against the oracle: the static droplet (EOS at the local T) in FP64 and
FP32 per-node-reference storage, a ragged walled lattice with gravity and
both wall conditions, the single-phase ideal-EOS cavity of Sec. III.B, and
switching treatments mid-run; the phi div u term of Eq. (5) in the
finite-difference and the LB treatments."""
import numpy as np
import pytest

from gpu_util import compare_fp32dev, compare_fp64, gpu_run, need_gpu, oracle_run, say
from oracle import CORRECTED, FD_RK2, PLAIN, Oracle
from paper_1405_2232_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


@pytest.mark.parametrize("precision", ["fp64", "fp32local"])
def test_droplet_fd_parity(precision):
    p, rho, T = inputs.static_droplet()
    say("case fd droplet", precision)
    g = gpu_run(p, rho, T, 2000, FD_RK2, precision=precision)
    o = oracle_run(p, rho, T, 2000, FD_RK2)
    if precision == "fp64":
        compare_fp64(g.moments(), o.moments(), what=("fd droplet",))
    else:
        compare_fp32dev(g.moments(), o.moments(), what=("fd droplet fp32local",))


def test_ragged_walls_gravity_fd_parity():
    Tc = inputs.cs_tc()
    p, rho, T = inputs.static_droplet(nx=77, ny=45, radius=12, seed=5)
    p.update(wall_x=True, wall_y=True, gy=-2e-5, thermal_left="adiabatic", thermal_right="dirichlet",
             thermal_bottom="dirichlet", thermal_top="adiabatic", T_right=0.88 * Tc,
             T_bottom=0.83 * Tc, eos_fixed_T=True)
    say("case fd ragged walls")
    g = gpu_run(p, rho, T, 500, FD_RK2)
    o = oracle_run(p, rho, T, 500, FD_RK2)
    compare_fp64(g.moments(), o.moments(), what=("fd ragged",))


def test_cavity_fd_parity():
    n = 40
    Th, Tl, mu, Pr, Ra = 1.03, 0.97, 0.1, 0.71, 1e3
    p = dict(nx=n, ny=n, tau_f=0.5 + 3 * mu, tau_g=0.5 + 3 * mu / Pr, G=1.0, beta=0.0, eos="ideal",
             R=1.0 / 3.0, cv=1.0, gx=0.0, gy=-Ra * mu ** 2 / ((Th - Tl) * n ** 3 * Pr), wall_x=True,
             wall_y=True, thermal_left="dirichlet", thermal_right="dirichlet", thermal_bottom="adiabatic",
             thermal_top="adiabatic", T_left=Th, T_right=Tl, eos_fixed_T=False, T_eos=1.0)
    one = np.ones((n, n))
    say("case fd cavity")
    g = gpu_run(p, one, one, 3000, FD_RK2)
    o = oracle_run(p, one, one, 3000, FD_RK2)
    compare_fp64(g.moments(), o.moments(), what=("fd cavity",))


def test_switching_treatments_mid_run():
    from paper_1405_2232_amd.lbm import Lattice
    p, rho, T = inputs.static_droplet(nx=48, ny=40, radius=10, seed=6)
    g = Lattice(p, "fp64")
    g.init_fields(rho, T)
    o = Oracle(p)
    o.init_fields(rho, T)
    for tr, k in ((CORRECTED, 100), (FD_RK2, 150), (CORRECTED, 80), (FD_RK2, 20)):
        g.step(k, tr)
        assert o.step(k, tr) == 0
    compare_fp64(g.moments(), o.moments(), what=("switching",))
    # the state itself: g = cv T f after a finite-difference step
    st = g.get_state()
    f, gg = o.get_state()
    assert np.abs(st[:9] - f).max() < 1e-12 and np.abs(st[9:] - gg).max() < 1e-12


@pytest.mark.parametrize("walls", [False, True])
def test_phi_divu_fd_parity(walls):
    Tc = inputs.cs_tc()
    p, rho, T = inputs.static_droplet(nx=70, ny=52, radius=13, seed=8)
    p["phi_divu"] = True
    if walls:
        p.update(wall_x=True, wall_y=True, thermal_left="adiabatic", thermal_right="dirichlet",
                 thermal_bottom="dirichlet", thermal_top="dirichlet", T_right=0.87 * Tc,
                 T_bottom=0.84 * Tc, T_top=0.86 * Tc, gy=-1e-5)
    say("case fd phi div u", walls)
    g = gpu_run(p, rho, T, 800, FD_RK2)
    o = oracle_run(p, rho, T, 800, FD_RK2)
    compare_fp64(g.moments(), o.moments(), what=("fd phi div u", walls))


@pytest.mark.parametrize("precision", ["fp64", "fp32local"])
@pytest.mark.parametrize("treatment", [CORRECTED, PLAIN])
@pytest.mark.parametrize("walls", [False, True])
def test_phi_divu_lb_parity(walls, treatment, precision):
    """The source w_i phi div u of Eq. (5) in the LB g update: GPU against
    the oracle on a two-phase droplet (EOS at T0 for the plain treatment,
    which otherwise leaves the EOS domain), periodic, and in a walled box
    with gravity and both wall conditions (a corner of each kind)."""
    Tc = inputs.cs_tc()
    p, rho, T = inputs.static_droplet(nx=70, ny=52, radius=13, seed=9)
    p["phi_divu"] = True
    p["eos_fixed_T"] = treatment == PLAIN
    if walls:
        p.update(wall_x=True, wall_y=True, thermal_left="adiabatic", thermal_right="dirichlet",
                 thermal_bottom="dirichlet", thermal_top="dirichlet", T_right=0.87 * Tc,
                 T_bottom=0.84 * Tc, T_top=0.86 * Tc, gy=-1e-5)
    say("case lb phi div u", walls, treatment, precision)
    g = gpu_run(p, rho, T, 800, treatment, precision=precision)
    assert not g.get_step_pairing()[0]
    o = oracle_run(p, rho, T, 800, treatment)
    if precision == "fp64":
        compare_fp64(g.moments(), o.moments(), what=("lb phi div u", walls, treatment))
    else:
        compare_fp32dev(g.moments(), o.moments(), what=("lb phi div u fp32local", walls, treatment))


def test_phi_divu_lb_open_channel_parity():
    """The source in the open channel's kernel variant (inlet and outlet of
    Sec. III.A), single-phase ideal gas with the beta = 0 force."""
    mu, Pr = 0.1, 0.71
    nx, ny = 90, 20
    p = dict(nx=nx, ny=ny, tau_f=0.5 + 3 * mu, tau_g=0.5 + 3 * mu / Pr, G=1.0, beta=0.0, eos="ideal",
             R=1.0 / 3.0, cv=1.0, gx=0.0, gy=0.0, wall_x="open", wall_y=True,
             thermal_left="dirichlet", thermal_right="adiabatic", thermal_bottom="dirichlet",
             thermal_top="dirichlet", T_left=1.03, T_bottom=0.97, T_top=0.97, u_in=0.05, rho_out=1.0,
             eos_fixed_T=False, T_eos=1.0, phi_divu=True)
    one = np.ones((ny, nx))
    say("case lb phi div u open channel")
    g = gpu_run(p, one, one, 1500, CORRECTED)
    o = oracle_run(p, one, one, 1500, CORRECTED)
    compare_fp64(g.moments(), o.moments(), what=("lb phi div u channel",))


def test_phi_divu_lattice_cannot_join_a_batch():
    from paper_1405_2232_amd.lbm import Batch, LbmError
    p, rho, T = inputs.static_droplet(nx=32, ny=32, radius=8, seed=1)
    q = dict(p, phi_divu=True)
    with pytest.raises(LbmError):
        Batch([p, q], "fp64")


@pytest.mark.parametrize("precision", ["fp64", "fp32local", "fp32dev"])
def test_fd_single_launch_step_equals_separate_passes(precision, monkeypatch):
    """A finite-difference step streams f and writes the moments of time t
    in one launch (two-row load look-ahead, the default); with a one-row
    look-ahead it takes a moments pass and a full step instead.  Both
    compute the same values, so the states agree bit for bit, on a ragged
    walled lattice with gravity."""
    from paper_1405_2232_amd.lbm import Lattice
    Tc = inputs.cs_tc()
    p, rho, T = inputs.static_droplet(nx=77, ny=45, radius=12, seed=5)
    p.update(wall_x=True, wall_y=True, gy=-2e-5, thermal_left="adiabatic", thermal_right="dirichlet",
             thermal_bottom="dirichlet", thermal_top="adiabatic", T_right=0.88 * Tc,
             T_bottom=0.83 * Tc, eos_fixed_T=True)
    say("case fd single launch", precision)
    states = []
    for pf in ("2", "1"):
        monkeypatch.setenv("LBM_PF", pf)
        g = Lattice(p, precision)
        g.init_fields(rho, T)
        g.step(300, FD_RK2)
        states.append(g.get_state())
        del g
    d = float(np.max(np.abs(states[0] - states[1])))
    say("max |d state|", d)
    assert np.array_equal(states[0], states[1])
