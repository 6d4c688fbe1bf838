"""Shared helpers of the GPU tests: run the same seeded input through the
HIP path and the oracle and compare."""
import sys

import numpy as np
import pytest

from oracle import Oracle

FP64_TOL = 1e-10          # max-abs on rho, u, T
FP32_RHO_REL = 2e-6       # max |d rho| / rho
FP32_T_ABS = 1e-5         # max |d T|


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def gpu_run(cfg, rho, T, steps, treatment, precision="fp64", ux=None, uy=None, tiling=None,
            chunks=None, pair=None):
    from paper_1405_2232_amd.lbm import Lattice
    g = Lattice(cfg, precision)
    g.init_fields(rho, T, ux, uy)
    if tiling is not None:
        g.set_tiling(*tiling)
    if pair is not None:
        g.set_step_pairing(pair)
    for n in (chunks or [steps]):
        if n > 0:
            g.step(n, treatment)
    return g


def oracle_run(cfg, rho, T, steps, treatment, ux=None, uy=None):
    o = Oracle(cfg)
    o.init_fields(rho, T, ux, uy)
    rc = o.step(steps, treatment)
    assert rc == 0, rc
    return o


def max_abs(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))))


def compare_fp64(mg, mo, tol=FP64_TOL, what=""):
    names = ("rho", "ux", "uy", "T")
    errs = {n: max_abs(a, b) for n, a, b in zip(names, mg, mo)}
    say("fp64 parity", what, errs)
    for n in names:
        assert np.all(np.isfinite(mg[names.index(n)])), n
        assert errs[n] <= tol, (what, n, errs)
    return errs


def compare_fp32dev(mg, mo, what=""):
    rho_rel = float(np.max(np.abs(mg[0] - mo[0]) / np.abs(mo[0])))
    T_abs = max_abs(mg[3], mo[3])
    u_abs = max(max_abs(mg[1], mo[1]), max_abs(mg[2], mo[2]))
    say("fp32dev error", what, dict(rho_rel=rho_rel, T_abs=T_abs, u_abs=u_abs))
    assert rho_rel <= FP32_RHO_REL, (what, rho_rel)
    assert T_abs <= FP32_T_ABS, (what, T_abs)
    return rho_rel, T_abs, u_abs
