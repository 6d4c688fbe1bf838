"""The learned warm start, end to end at a small size: solver trajectories
(FP64 LB, run to a one-step residual target) train the network on the GPU
with its own kernels; on held-out cases the warm start (prediction
screened by its own residual, cold start where rejected) must reach the
target in fewer LB steps than the cold start, and end in the same steady
state."""
import numpy as np
import pytest

from gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu

N = 64
TARGET = 1e-7
CAP = 120000


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def test_warm_start_needs_fewer_steps_than_cold_start():
    from paper_1405_2232_amd import inputs
    from paper_1405_2232_amd.warmstart import WarmStart, screen, solve
    train = [inputs.warmstart_case(s, n=N, max_drops=3) for s in range(48)]
    test = [inputs.warmstart_case(200000 + s, n=N, max_drops=3) for s in range(12)]
    r = solve(train, target=TARGET, cap=CAP)
    keep = [i for i, s in enumerate(r["steps"]) if s is not None]
    say("training solves converged", len(keep), "of", len(train), "mean steps",
        float(np.mean([r["steps"][i] for i in keep])) if keep else None)
    assert len(keep) >= 24
    ws = WarmStart(N)
    data = ws.dataset([train[i] for i in keep], [r["fields"][i] for i in keep])
    hist = ws.train(data, epochs=25, lr=2e-3)
    say("loss first/last epoch", hist[0], hist[-1])
    assert hist[-1] < 0.5 * hist[0]
    cold = solve(test, target=TARGET, cap=CAP)
    preds = ws.predict(test)
    inits = screen(test, preds)
    warm = solve(test, inits=inits, target=TARGET, cap=CAP)
    both = [i for i in range(len(test)) if cold["steps"][i] is not None and warm["steps"][i] is not None]
    cs = sum(cold["steps"][i] for i in both)
    wsum = sum(warm["steps"][i] for i in both)
    say("held-out: accepted", sum(p is not None for p in inits), "converged cold/warm",
        sum(s is not None for s in cold["steps"]), sum(s is not None for s in warm["steps"]),
        "steps cold", cs, "warm", wsum)
    assert len(both) >= len(test) // 2
    assert wsum < cs
    # both starts must end in the same steady state
    for i in both:
        dr = float(np.mean(np.abs(warm["fields"][i][0] - cold["fields"][i][0])))
        dT = float(np.max(np.abs(warm["fields"][i][1] - cold["fields"][i][1])))
        say("case", i, "steady-state difference warm vs cold: mean |d rho|", dr, "max |d T|", dT)
        assert dr < 1e-3 and dT < 1e-4
