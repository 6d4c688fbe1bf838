"""The learned warm start against the method without it.

The network weights are the ones `python -m
paper_1405_2232_amd.train_warmstart --physical` wrote from FP64 solver
trajectories started at rest in the forcing scheme's velocity (seeds
0..3999, the converged ones) with the library's own training kernels.  On
held-out cases (seeds 200000..) both solves start that way (stored momentum
-F/2, the best start without the network): the warm start replaces only the
initial density and temperature by the network's mass-conserving
prediction, kept when its one-step residual is not above the cold start's.
Checked: the screen keeps only such predictions; the warm start converges
at least as often and takes fewer steps in all; both reach the same steady
state (compared pointwise after the rigid translation between them: a
droplet at rest may settle anywhere along the periodic x, and anywhere in
y while clear of the walls); and the steps and wall time of both are
reported."""
import os

import numpy as np
import pytest

from gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu

N = 64
TARGET = 1e-7
CAP = 400000
WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_1405_2232_amd", "warmstart_64.npz")


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _peak(cc):
    """Position of the maximum of a periodic sequence, refined by the
    parabola through it and its two neighbours."""
    k, n = int(np.argmax(cc)), len(cc)
    y0, y1, y2 = cc[(k - 1) % n], cc[k], cc[(k + 1) % n]
    return k + 0.5 * (y0 - y2) / (y0 - 2.0 * y1 + y2)


def _translate(b, s, axis):
    """b moved by s nodes (any real s) along an axis, by a Fourier phase ramp."""
    ph = np.exp(-2j * np.pi * np.fft.fftfreq(b.shape[axis]) * s)
    ph = ph[None, :] if axis == 1 else ph[:, None]
    return np.fft.ifft(np.fft.fft(b, axis=axis) * ph, axis=axis).real


def _align(a, b):
    """The rigid translation (sx, sy) of b that best matches a: the peaks of
    the cross-correlations of column means (x) and then of row means (y).
    A droplet at rest is free to settle anywhere along the periodic x, and
    anywhere in y while it keeps clear of the walls."""
    ma, mb = a.mean(axis=0) - a.mean(), b.mean(axis=0) - b.mean()
    sx = _peak(np.fft.ifft(np.fft.fft(ma) * np.conj(np.fft.fft(mb))).real)
    b1 = _translate(b, sx, 1)
    ra, rb = a.mean(axis=1) - a.mean(), b1.mean(axis=1) - b1.mean()
    sy = _peak(np.fft.ifft(np.fft.fft(ra) * np.conj(np.fft.fft(rb))).real)
    sy = sy - len(ra) if sy > len(ra) / 2 else sy
    return sx, sy


def test_warm_start_against_physical_cold_start():
    from paper_1405_2232_amd import inputs
    from paper_1405_2232_amd.warmstart import WarmStart, load_params, screen, solve
    assert os.path.exists(WEIGHTS), "trained weights missing: " + WEIGHTS
    test = [inputs.warmstart_case(200000 + s, n=N, max_drops=3) for s in range(16)]
    ws = WarmStart(N, params=load_params(WEIGHTS))
    preds = ws.predict(test)
    for (p, rho, T), (pr, pt) in zip(test, preds):
        assert abs(pr.sum() - rho.sum()) <= 1e-9 * rho.sum()
    inits, rp, rc = screen(test, preds, physical=True)
    for kept, a, b in zip(inits, rp, rc):
        assert kept is None or a <= b or a <= 1e-3
    cold = solve(test, target=TARGET, cap=CAP, physical=True)
    warm = solve(test, inits=inits, target=TARGET, cap=CAP, physical=True)
    cs = sum(s if s is not None else CAP for s in cold["steps"])
    wsum = sum(s if s is not None else CAP for s in warm["steps"])
    nc = sum(s is not None for s in cold["steps"])
    nw = sum(s is not None for s in warm["steps"])
    say("accepted", sum(p is not None for p in inits), "of", len(test), "converged cold/warm", nc, nw,
        "steps (unconverged at the cap) cold", cs, "warm", wsum,
        "wall s cold %.2f warm %.2f" % (cold["wall_s"], warm["wall_s"]))
    # the gain: at least as many converged solves, and fewer steps in all
    # (unconverged solves counted at the cap)
    assert nw >= nc
    assert wsum < cs
    # the same steady state: both solves stop at a one-step residual r
    # while the slowest mode (a decade of r per ~1e5 steps, e-folding over
    # tau ~ 4e4 steps) still moves the fields by up to ~ r tau ~ 4e-3
    # relative; compared pointwise after the rigid translation between them
    both = [i for i in range(len(test)) if cold["steps"][i] is not None and warm["steps"][i] is not None]
    for i in both:
        rw, rc_ = warm["fields"][i][0], cold["fields"][i][0]
        tw, tc = warm["fields"][i][1], cold["fields"][i][1]
        sx, sy = _align(rc_, rw)
        rwa = _translate(_translate(rw, sx, 1), sy, 0)
        twa = _translate(_translate(tw, sx, 1), sy, 0)
        dr = float(np.mean(np.abs(rwa - rc_) / rc_))
        dT = float(np.mean(np.abs(twa - tc) / tc))
        say("case", i, "shift x %.3f y %.3f" % (sx, sy), "mean |d rho|/rho", dr, "mean |d T|/T", dT,
            "max |d rho|/rho", float(np.max(np.abs(rwa - rc_) / rc_)))
        assert dr < 4e-3 and dT < 4e-3
