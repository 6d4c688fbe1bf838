"""lbm_totals_noalloc (the totals with the library's static scratch array
instead of the workspace's) against lbm_totals, through the C ABI: two
calls in a row on one GPU, the second on a smaller lattice, then the first
lattice again; the results must be equal bit for bit (same kernels, same
fixed reduction order)."""
import numpy as np
import pytest

from gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


def _lattice(nx, ny, precision, steps, seed):
    from paper_1405_2232_amd import inputs
    from paper_1405_2232_amd.lbm import CORRECTED, Lattice
    p, rho, T = inputs.static_droplet(nx=nx, ny=ny, radius=0.3 * min(nx, ny), seed=seed)
    p.update(wall_y=True, T_bottom=0.84 * inputs.cs_tc(), T_top=0.88 * inputs.cs_tc(), gy=-1e-5)
    g = Lattice(p, precision)
    g.init_fields(rho, T)
    g.step(steps, CORRECTED)
    return g


def test_totals_noalloc_equals_totals_second_call_smaller():
    need_gpu()
    big = _lattice(1000, 700, "fp32local", 40, 3)    # 4 x 88 moments blocks
    small = _lattice(90, 50, "fp64", 30, 4)          # 2 x 7
    for what, g in (("1000x700 fp32local", big), ("90x50 fp64", small), ("1000x700 again", big)):
        say("totals_noalloc", what)
        a = g.totals()
        b = g.totals_noalloc()
        say(" ", a.tolist(), b.tolist())
        assert np.isfinite(a[:5]).all()
        assert a[0] > 0 and a[1] > 0
        assert np.array_equal(a, b), (what, a, b)


def test_totals_noalloc_state_and_size_limits():
    need_gpu()
    from paper_1405_2232_amd import inputs
    from paper_1405_2232_amd.lbm import ESTATE, EINVAL, Lattice, LbmError
    # not initialised
    p, rho, T = inputs.static_droplet(nx=32, ny=32, radius=8, seed=1)
    g = Lattice(p, "fp64", rho_ref=1.0, T_ref=1.0)
    g._create(None, None)
    with pytest.raises(LbmError) as e:
        g.totals_noalloc()
    assert e.value.status == ESTATE
    # a moments launch of 32769 blocks (1 x 262152 nodes: one 62-column
    # strip, 8-row bands) is beyond the static array
    ny = 8 * 32769
    p = inputs.base_params(1, ny, 0.08)
    p.update(G=0.0)
    g = Lattice(p, "fp32local", rho_ref=1.0, T_ref=1.0)
    g.init_fields(np.ones((ny, 1)), np.ones((ny, 1)))
    with pytest.raises(LbmError) as e:
        g.totals_noalloc()
    assert e.value.status == EINVAL
    assert np.isfinite(g.totals()[0])
