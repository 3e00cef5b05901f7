"""Parity of the coarse Re_tau 640 channel (128 x 64 x 64, FP32 storage and
arithmetic, WFB and bounce-back walls, plane statistics accumulated in FP64
on every step: the time and plane averages of Sec. 3.1 behind the profiles of
Fig. 6) against the FP64 oracle after 200 steps, element by element for the
velocity field and layer by layer for the statistics.

Tolerance, from the arithmetic: each step the FP32 path rounds every stored
population once (half an FP32 ulp of |h| <= 0.1 is below 3e-9) and computes
in FP32 (the one-step bound of the kernel arithmetic, 2e-8).  Without
amplification these errors add up over N steps; the velocity sums ten
populations with e_x != 0 (divided by rho ~ 1), so
    |du| <= N * 10 * (3e-9 + 2e-8) = N * 2.3e-7.
The statistics inherit the same bound for the layer means of u and
2 |u|max |du| + |du|^2 for the second moments."""
import numpy as np
import pytest

from gpu_common import oracle_for

pytestmark = pytest.mark.gpu

STEPS = 200
PER_STEP = 10 * (3e-9 + 2e-8)


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_04352_amd as P
    return P


@pytest.mark.parametrize("bc", ("wfb", "bb"))
def test_c2_fp32_200_steps_with_statistics(P, orc, bc):
    from paper_2009_04352_amd import workloads as W
    print("c2 FP32 %s %d steps" % (bc, STEPS), flush=True)
    p = W.params("c2")
    nx, ny, nz = p["grid"]
    ch = P.Channel(nx, ny, nz, p["tau0"], cs=p["cs"], fx=p["fx"], store="f32", bc=bc, stats_every=1,
                   tiles=W.launch_tiles("c2", "f32"))
    o = oracle_for(orc, p["grid"], p["tau0"], p["cs"], p["fx"], bc, stats_every=1)
    ch.init_spalding(p["u_tau"], p["noise"], p["seed"])
    o.init_spalding(p["u_tau"], p["noise"], p["seed"])
    ch.step(STEPS)
    assert o.step(STEPS) == 0
    assert ch.sync()[0] == 0
    tol_u = STEPS * PER_STEP
    rg, xg, yg, zg = ch.moments()
    ro, xo, yo, zo = o.observe()
    du = max(np.abs(xg - xo).max(), np.abs(yg - yo).max(), np.abs(zg - zo).max())
    print("max|du|/u_tau = %.3e (bound %.3e)" % (du / p["u_tau"], tol_u / p["u_tau"]), flush=True)
    assert du <= tol_u
    assert np.abs(rg - ro).max() <= STEPS * 19 * (3e-9 + 2e-8)
    # FP64 plane statistics: sample counts exact, layer means and second moments within the bound
    sg, ng = ch.stats_sums()
    so, no = o.stats_sums()
    assert ng == no == STEPS
    np.testing.assert_array_equal(sg[:, 7], so[:, 7])
    m = so[:, 7:8]
    umax = max(np.abs(xo).max(), np.abs(yo).max(), np.abs(zo).max()) * 1.5
    np.testing.assert_allclose(sg[:, 0:3] / m, so[:, 0:3] / m, rtol=0, atol=tol_u)
    np.testing.assert_allclose(sg[:, 3:7] / m, so[:, 3:7] / m, rtol=0, atol=2 * umax * tol_u + tol_u ** 2)
    ch.close()
