"""Two steps per launch (temporal blocking) against one-step launches and
against the FP64 oracle.

The two-step kernel runs the one-step kernel's arithmetic on the same
stored values (FP32 or FP64), so pairing steps must leave the state bit for bit
unchanged, and the result must meet the FP32 parity bar against the
oracle.  Cases span several strips and bands with ragged tails, y walls
(Dirichlet and adiabatic), gravity, odd step counts (a one-step launch at
the end), periodic checks falling between pairs, and lattices narrower or
shorter than one tile."""
import numpy as np
import pytest

from gpu_util import compare_fp32dev, compare_fp64, need_gpu, oracle_run, say
from oracle import CORRECTED, PLAIN
from paper_1405_2232_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _run(p, rho, T, steps, tr, precision, pair, rows=0, check=0, chunks=None):
    from paper_1405_2232_amd.lbm import Lattice
    g = Lattice(p, precision)
    g.init_fields(rho, T)
    g.set_step_pairing(pair, rows)
    if check:
        g.set_check_interval(check)
    for n in (chunks or [steps]):
        g.step(n, tr)
    return g


def _cases():
    Tc = inputs.cs_tc()
    out = []
    p, rho, T = inputs.static_droplet()
    out.append(("64x64 droplet", p, rho, T, 301, CORRECTED))
    p, rho, T = inputs.static_droplet()
    p["eos_fixed_T"] = True
    out.append(("64x64 droplet plain fixed-T", p, rho, T, 300, PLAIN))
    p, rho, T = inputs.static_droplet(nx=300, ny=70, radius=15, seed=11)
    p.update(wall_y=True, T_bottom=0.8 * Tc, T_top=0.9 * Tc, gy=-2e-5)
    out.append(("300x70 walls+gravity", p, rho, T, 301, CORRECTED))
    p, rho, T = inputs.static_droplet(nx=520, ny=33, radius=10, seed=13)
    p.update(wall_y=True, thermal_bottom="adiabatic", thermal_top="dirichlet", T_top=0.9 * Tc,
             gx=1e-5)
    out.append(("520x33 adiabatic bottom", p, rho, T, 150, CORRECTED))
    p, rho, T = inputs.static_droplet(nx=37, ny=23, radius=7, seed=12)
    p["eos_fixed_T"] = True
    out.append(("37x23 periodic plain", p, rho, T, 201, PLAIN))
    p, rho, T = inputs.static_droplet(nx=1, ny=48, radius=10, seed=14)
    out.append(("1x48", p, rho, T, 200, CORRECTED))
    p, rho, T = inputs.static_droplet(nx=48, ny=1, radius=10, seed=15)
    out.append(("48x1", p, rho, T, 200, CORRECTED))
    p, rho, T = inputs.static_droplet(nx=20, ny=5, radius=3, seed=17)
    p.update(wall_y=True, T_bottom=0.8 * Tc, T_top=0.9 * Tc)
    out.append(("20x5 walls", p, rho, T, 99, CORRECTED))
    # the mixed force of Eq. (4)
    p, rho, T = inputs.static_droplet(nx=260, ny=45, radius=10, seed=13)
    p.update(beta=0.5, gx=1e-5, wall_y=True, T_bottom=0.8 * Tc, T_top=0.9 * Tc)
    out.append(("260x45 beta=0.5 walls", p, rho, T, 151, CORRECTED))
    # ideal EOS with beta = 0 (the model of the paper's Section III),
    # periodic in x
    n = 50
    x = np.arange(n)[None, :]
    rho = np.ones((40, n)) * (1.0 + 0.01 * np.sin(2 * np.pi * x / n))
    T = np.ones((40, n)) * (1.0 + 0.03 * np.cos(2 * np.pi * x / n))
    p = dict(nx=n, ny=40, tau_f=0.8, tau_g=0.5 + 0.3 / 0.71, G=1.0, beta=0.0, eos="ideal",
             R=1.0 / 3.0, cv=1.0, wall_y=True, thermal_bottom="dirichlet", thermal_top="adiabatic",
             T_bottom=1.03, gy=-1e-4)
    out.append(("50x40 ideal beta=0", p, rho, T, 200, PLAIN))
    return out


@pytest.mark.parametrize("precision", ["fp32local", "fp32dev", "fp64"])
@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
def test_pairs_equal_single_steps(case, precision):
    name, p, rho, T, steps, tr = case
    say("case pair", name, precision, steps)
    a = _run(p, rho, T, steps, tr, precision, pair=False)
    b = _run(p, rho, T, steps, tr, precision, pair=True)
    assert b.get_step_pairing()[0]
    sa, sb = a.get_state(), b.get_state()
    d = float(np.max(np.abs(sa - sb)))
    say("pair vs single max |d state|", name, precision, d)
    assert np.array_equal(sa, sb), (name, d)
    ta, tb = a.totals(), b.totals()
    assert ta[5] == tb[5] and ta[6] == tb[6] == steps
    if precision == "fp32local":
        o = oracle_run(p, rho, T, steps, tr)
        compare_fp32dev(b.moments(), o.moments(), what=("pair", name))
    if precision == "fp64":
        o = oracle_run(p, rho, T, steps, tr)
        compare_fp64(b.moments(), o.moments(), what=("pair", name))


def test_pair_rows_invariance():
    Tc = inputs.cs_tc()
    p, rho, T = inputs.static_droplet(nx=150, ny=90, radius=20, seed=21)
    p.update(wall_y=True, T_bottom=0.8 * Tc, T_top=0.9 * Tc)
    ref = None
    for rows in (8, 1, 3, 16, 90):
        say("case pair rows", rows)
        s = _run(p, rho, T, 60, CORRECTED, "fp32local", pair=True, rows=rows).get_state()
        if ref is None:
            ref = s
        else:
            assert np.array_equal(s, ref), rows


def test_pair_with_checks_and_chunks():
    """Periodic checks between pairs and odd chunk lengths keep the state
    and the step count of one-step launches."""
    p, rho, T = inputs.static_droplet(seed=5)
    a = _run(p, rho, T, 0, CORRECTED, "fp32local", pair=False, chunks=[157])
    b = _run(p, rho, T, 0, CORRECTED, "fp32local", pair=True, check=7, chunks=[3, 50, 1, 103])
    assert np.array_equal(a.get_state(), b.get_state())
    assert b.totals()[6] == 157


def test_pair_clamp_count():
    """The plain treatment with the EOS at the local T leaves the real-psi
    domain after a few tens of steps: the clamp count (first and second step
    of each pair) equals the one-step count."""
    p, rho, T = inputs.static_droplet()
    a = _run(p, rho, T, 80, PLAIN, "fp32local", pair=False)
    b = _run(p, rho, T, 80, PLAIN, "fp32local", pair=True)
    ca, cb = a.totals()[5], b.totals()[5]
    say("clamps single", ca, "pair", cb)
    assert ca > 0 and ca == cb
    assert np.array_equal(a.get_state(), b.get_state())


def test_pair_eligibility():
    from paper_1405_2232_amd.lbm import Lattice
    p, rho, T = inputs.static_droplet(nx=32, ny=32, radius=8, seed=1)
    for prec, extra, want in (("fp32local", {}, True), ("fp32dev", {}, True), ("fp64", {}, True),
                              ("fp32local", {"wall_x": True}, False),
                              ("fp32local", {"beta": 0.5}, True),
                              ("fp32local", {"G": 0.0, "beta": 0.5}, True)):
        g = Lattice(dict(p, **extra), prec)
        g.init_fields(rho, T)
        assert not g.get_step_pairing()[0]  # too small to pair by default
        g.set_step_pairing(True)
        assert g.get_step_pairing()[0] == want, (prec, extra)
        g.set_step_pairing(False)
        assert not g.get_step_pairing()[0]


@pytest.mark.parametrize("bx", ["64", "128", "256"])
def test_pair_block_widths(bx, monkeypatch):
    """Every block width of the two-step kernel (64, 128 or 256 lanes;
    6 halo columns each) gives the one-step result bit for bit."""
    monkeypatch.setenv("LBM_PAIR_BX", bx)
    Tc = inputs.cs_tc()
    p, rho, T = inputs.static_droplet(nx=300, ny=70, radius=15, seed=11)
    p.update(wall_y=True, T_bottom=0.8 * Tc, T_top=0.9 * Tc, gy=-2e-5)
    a = _run(p, rho, T, 41, CORRECTED, "fp32local", pair=False)
    for rows in (0, 5):
        say("case pair bx", bx, "rows", rows)
        b = _run(p, rho, T, 41, CORRECTED, "fp32local", pair=True, rows=rows)
        assert np.array_equal(a.get_state(), b.get_state()), (bx, rows)


def test_pair_full_size_wall_slab_bitwise():
    """The benchmark's lattice and launch shape (2048 x 2048 wall slab,
    default two-step tiling, periodic checks every 100 steps): 201 steps
    paired give the one-step launches' state bit for bit."""
    p, rho, T = inputs.wall_slab()
    a = _run(p, rho, T, 201, CORRECTED, "fp32local", pair=False, check=100)
    b = _run(p, rho, T, 201, CORRECTED, "fp32local", pair=True, check=100)
    say("full-size pairing", b.get_step_pairing())
    for x, y in zip(a.moments(), b.moments()):
        assert np.array_equal(x, y)
    assert np.array_equal(a.get_state(), b.get_state())
