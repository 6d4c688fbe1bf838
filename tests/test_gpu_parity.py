"""GPU parity: the HIP path against the FP64 oracle, element by element, on
the same seeded inputs, through the C ABI."""
import numpy as np
import pytest

from gpu_util import (FP64_TOL, compare_fp32dev, compare_fp64, gpu_run, max_abs, need_gpu,
                      oracle_run, say)
from oracle import CORRECTED, PLAIN, Oracle
from paper_1405_2232_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


# ---------------------------------------------------------------------------
# 64 x 64 static droplet, 2000 steps, both treatments
# ---------------------------------------------------------------------------

DROPLET_CASES = [
    # (treatment, EOS at fixed T0, steps)
    (PLAIN, True, 2000),
    (CORRECTED, True, 2000),
    (CORRECTED, False, 2000),
    # with the EOS at the local T the plain equation leaves the real-psi
    # domain after ~35 steps; its parity is checked before that
    (PLAIN, False, 30),
]


@pytest.mark.parametrize("treatment,fixed,steps", DROPLET_CASES)
def test_droplet_fp64_parity(treatment, fixed, steps):
    p, rho, T = inputs.static_droplet()
    p["eos_fixed_T"] = fixed
    say("case droplet fp64", treatment, fixed, steps)
    g = gpu_run(p, rho, T, steps, treatment)
    o = oracle_run(p, rho, T, steps, treatment)
    compare_fp64(g.moments(), o.moments(), what=("droplet", treatment, fixed, steps))


@pytest.mark.parametrize("treatment,fixed,steps", DROPLET_CASES)
def test_droplet_fp32local_parity(treatment, fixed, steps):
    p, rho, T = inputs.static_droplet()
    p["eos_fixed_T"] = fixed
    say("case droplet fp32local", treatment, fixed, steps)
    g = gpu_run(p, rho, T, steps, treatment, precision="fp32local")
    o = oracle_run(p, rho, T, steps, treatment)
    compare_fp32dev(g.moments(), o.moments(), what=("droplet fp32local", treatment, fixed, steps))


@pytest.mark.parametrize("treatment,fixed,steps", DROPLET_CASES)
def test_droplet_fp32dev_global_error(treatment, fixed, steps):
    """The global-shift FP32 form: its error against the oracle is stated,
    and bounded by a looser limit (temperature still within 1e-5)."""
    p, rho, T = inputs.static_droplet()
    p["eos_fixed_T"] = fixed
    say("case droplet fp32dev", treatment, fixed, steps)
    g = gpu_run(p, rho, T, steps, treatment, precision="fp32dev")
    o = oracle_run(p, rho, T, steps, treatment)
    mg, mo = g.moments(), o.moments()
    rho_rel = float(np.max(np.abs(mg[0] - mo[0]) / mo[0]))
    T_abs = max_abs(mg[3], mo[3])
    say("fp32dev global error", (treatment, fixed, steps), dict(rho_rel=rho_rel, T_abs=T_abs))
    assert rho_rel < 1e-4 and T_abs < 1e-5


# ---------------------------------------------------------------------------
# ragged sizes, several tiles, walls, gravity, mixed force, ideal EOS
# ---------------------------------------------------------------------------

def _ragged_cases():
    Tc = inputs.cs_tc()
    cases = []
    # several strips and bands with a ragged tail, walls in y, gravity
    p, rho, T = inputs.static_droplet(nx=300, ny=70, radius=15, seed=11)
    p.update(wall_y=True, T_bottom=0.8 * Tc, T_top=0.9 * Tc, gy=-2e-5)
    cases.append(("300x70 walls+gravity", p, rho, T, 300, CORRECTED))
    p, rho, T = inputs.static_droplet(nx=37, ny=23, radius=7, seed=12)
    p["eos_fixed_T"] = True
    cases.append(("37x23 periodic plain", p, rho, T, 200, PLAIN))
    p, rho, T = inputs.static_droplet(nx=520, ny=33, radius=10, seed=13)
    p.update(beta=0.5, gx=1e-5)
    cases.append(("520x33 beta=0.5", p, rho, T, 150, CORRECTED))
    # single row / single column lattices
    p, rho, T = inputs.static_droplet(nx=1, ny=48, radius=10, seed=14)
    cases.append(("1x48", p, rho, T, 200, CORRECTED))
    p, rho, T = inputs.static_droplet(nx=48, ny=1, radius=10, seed=15)
    cases.append(("48x1", p, rho, T, 200, CORRECTED))
    # walls all round, Dirichlet sides, adiabatic top and bottom
    p, rho, T = inputs.static_droplet(nx=45, ny=40, radius=9, seed=16)
    p.update(wall_x=True, wall_y=True, thermal_left="dirichlet", thermal_right="dirichlet",
             thermal_bottom="adiabatic", thermal_top="adiabatic", T_left=0.82 * Tc,
             T_right=0.88 * Tc, gy=-1e-5)
    cases.append(("45x40 box", p, rho, T, 300, CORRECTED))
    # ideal EOS with beta = 0 (the model of the paper's Section III)
    n = 50
    x = np.arange(n)[None, :]
    rho = np.ones((40, n)) * (1.0 + 0.01 * np.sin(2 * np.pi * x / n))
    T = np.ones((40, n)) * (1.0 + 0.03 * np.cos(2 * np.pi * x / n))
    p = dict(nx=n, ny=40, tau_f=0.8, tau_g=0.5 + 0.3 / 0.71, G=1.0, beta=0.0, eos="ideal",
             R=1.0 / 3.0, cv=1.0, wall_x=True, wall_y=True, thermal_left="dirichlet",
             thermal_right="dirichlet", thermal_bottom="adiabatic", thermal_top="adiabatic",
             T_left=1.03, T_right=0.97, gy=-1e-4)
    cases.append(("ideal beta=0 cavity", p, rho, T, 300, PLAIN))
    cases.append(("ideal beta=0 cavity corrected", dict(p), rho, T, 300, CORRECTED))
    return cases


@pytest.mark.parametrize("case", _ragged_cases(), ids=lambda c: c[0])
def test_ragged_fp64_parity(case):
    name, p, rho, T, steps, tr = case
    say("case ragged fp64", name)
    g = gpu_run(p, rho, T, steps, tr)
    o = oracle_run(p, rho, T, steps, tr)
    compare_fp64(g.moments(), o.moments(), what=name)


@pytest.mark.parametrize("case", _ragged_cases(), ids=lambda c: c[0])
def test_ragged_fp32local_parity(case):
    name, p, rho, T, steps, tr = case
    say("case ragged fp32local", name)
    g = gpu_run(p, rho, T, steps, tr, precision="fp32local")
    o = oracle_run(p, rho, T, steps, tr)
    compare_fp32dev(g.moments(), o.moments(), what=name)


# ---------------------------------------------------------------------------
# tiling does not change the arithmetic; conservation; checkpoints
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("precision", ["fp64", "fp32dev", "fp32local"])
def test_tiling_invariance_bitwise(precision):
    Tc = inputs.cs_tc()
    p, rho, T = inputs.static_droplet(nx=150, ny=90, radius=20, seed=21)
    p.update(wall_y=True, T_bottom=0.8 * Tc, T_top=0.9 * Tc)
    ref = None
    for tiling in (None, (64, 1), (128, 3), (256, 7), (512, 5), (64, 90)):
        say("case tiling", precision, tiling)
        g = gpu_run(p, rho, T, 60, CORRECTED, precision=precision, tiling=tiling, pair=False)
        s = g.get_state()
        if ref is None:
            ref = s
        else:
            assert np.array_equal(s, ref), tiling


def test_totals_and_conservation():
    p, rho, T = inputs.static_droplet()
    p["eos_fixed_T"] = True
    g = gpu_run(p, rho, T, 0, CORRECTED, chunks=[0])
    t0 = g.totals()
    g.step(1000, CORRECTED)
    t1 = g.totals()
    o = oracle_run(p, rho, T, 1000, CORRECTED)
    to = o.totals()
    say("totals gpu", t1, "oracle", to)
    assert abs(t1[0] - t0[0]) < 1e-12 * t0[0]
    assert abs(t1[1] - t0[1]) < 1e-12 * t0[1]
    assert abs(t1[0] - to[0]) < 1e-12 * to[0]
    assert abs(t1[2] - to[2]) < 1e-12 and abs(t1[3] - to[3]) < 1e-12
    assert t1[4] == 0 and t1[5] == 0 and t1[6] == 1000


@pytest.mark.parametrize("precision", ["fp64", "fp32dev", "fp32local"])
def test_checkpoint_resume_bitwise(precision, tmp_path):
    p, rho, T = inputs.static_droplet(seed=3)
    g = gpu_run(p, rho, T, 100, CORRECTED, precision=precision)
    path = str(tmp_path / "ck.bin")
    g.save(path)
    g.step(150, CORRECTED)
    a = g.get_state()
    ta = g.totals()
    h = gpu_run(p, rho, T, 0, CORRECTED, precision=precision, chunks=[0])
    h.load(path)
    h.step(150, CORRECTED)
    assert np.array_equal(h.get_state(), a)
    assert h.totals()[6] == ta[6] == 250


@pytest.mark.parametrize("precision", ["fp32dev", "fp32local"])
def test_checkpoint_rejects_other_deviation_shifts(precision, tmp_path):
    """The FP32 forms store deviations from w_i rho_ref and w_i rho cv T_ref:
    a checkpoint loads only into a handle with the same shifts (LBM_EINVAL
    otherwise, and the handle's state is left as it was)."""
    from paper_1405_2232_amd.lbm import EINVAL, Lattice, LbmError
    p, rho, T = inputs.static_droplet(seed=3)
    g = Lattice(p, precision, rho_ref=float(rho.mean()), T_ref=float(T.mean()))
    g.init_fields(rho, T)
    g.step(20, CORRECTED)
    path = str(tmp_path / "ck.bin")
    g.save(path)
    for rr, tr in ((float(rho.mean()), 1.01 * float(T.mean())), (1.02 * float(rho.mean()), float(T.mean()))):
        if precision == "fp32local" and rr != float(rho.mean()):
            continue  # the per-node form has no global density shift
        h = Lattice(p, precision, rho_ref=rr, T_ref=tr)
        h.init_fields(rho, T)
        before = h.get_state()
        with pytest.raises(LbmError) as e:
            h.load(path)
        assert e.value.status == EINVAL
        assert np.array_equal(h.get_state(), before)
    same = Lattice(p, precision, rho_ref=float(rho.mean()), T_ref=float(T.mean()))
    same.init_fields(rho, T)
    same.load(path)
    assert np.array_equal(same.get_state(), g.get_state())


@pytest.mark.parametrize("precision", ["fp64", "fp32dev", "fp32local"])
def test_state_roundtrip(precision):
    """get_state/set_state is the FP64 view; for FP64 storage it is exact."""
    p, rho, T = inputs.static_droplet(seed=6)
    g = gpu_run(p, rho, T, 40, CORRECTED, precision=precision)
    s = g.get_state()
    h = gpu_run(p, rho, T, 0, CORRECTED, precision=precision, chunks=[0])
    h.set_state(s)
    s2 = h.get_state()
    tol = 0.0 if precision == "fp64" else 1e-8
    assert max_abs(s2, s) <= tol


def test_state_matches_oracle_distributions():
    p, rho, T = inputs.static_droplet(nx=40, ny=30, radius=8, seed=4)
    g = gpu_run(p, rho, T, 50, CORRECTED)
    o = oracle_run(p, rho, T, 50, CORRECTED)
    f, gg = o.get_state()
    s = g.get_state()
    assert max_abs(s[:9], f) < FP64_TOL
    assert max_abs(s[9:], gg) < FP64_TOL


def test_step_residual_matches_oracle():
    p, rho, T = inputs.static_droplet(seed=5)
    g = gpu_run(p, rho, T, 200, CORRECTED)
    r_gpu = g.step_residual(CORRECTED)
    o = oracle_run(p, rho, T, 200, CORRECTED)
    r0, _, _, T0 = o.moments()
    o.step(1, CORRECTED)
    r1, _, _, T1 = o.moments()
    r_ref = max(np.abs(r1 - r0).max() / np.abs(r1).max(), np.abs(T1 - T0).max() / np.abs(T1).max())
    say("residual", r_gpu, r_ref)
    assert r_gpu == pytest.approx(r_ref, rel=1e-5)


# ---------------------------------------------------------------------------
# status reporting
# ---------------------------------------------------------------------------

def test_nonfinite_detected_by_periodic_check():
    """The coupled plain case diverges on its own (no planted fault): the
    periodic check turns it into LBM_ENONFINITE."""
    from paper_1405_2232_amd import lbm
    p, rho, T = inputs.static_droplet()
    g = gpu_run(p, rho, T, 0, PLAIN, chunks=[0])
    g.set_check_interval(10)
    rc = g.step(300, PLAIN, check=False)
    assert rc == lbm.ENONFINITE
    o = Oracle(p)
    o.init_fields(rho, T)
    o.step(300, PLAIN)
    assert not np.all(np.isfinite(o.moments()[0]))


def test_psi_domain_policy_and_clamp_count():
    from paper_1405_2232_amd import lbm
    n = 16
    p = inputs.base_params(n, n, 0.08)
    rho = np.full((n, n), 0.03)
    T = np.full((n, n), 0.08)
    T[4:8, 4:8] = 0.5
    g = gpu_run(p, rho, T, 1, CORRECTED)
    o = oracle_run(p, rho, T, 1, CORRECTED)
    assert g.totals()[5] == o.totals()[5] >= 16
    p["psi_policy"] = 1
    g = gpu_run(p, rho, T, 1, CORRECTED)
    assert g.sync() == lbm.EDOMAIN


def test_bad_inputs_rejected():
    from paper_1405_2232_amd import lbm
    p, rho, T = inputs.static_droplet()
    bad = rho.copy()
    bad[3, 4] = np.nan
    g = lbm.Lattice(p)
    with pytest.raises(lbm.LbmError) as e:
        g.init_fields(bad, T)
    assert e.value.status == lbm.EINVAL
