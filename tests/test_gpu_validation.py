"""The wall-law validation path (Sec. 3.2: plane statistics of the time and
plane averages, Eq. 19 error norms against Spalding's law, Eq. 20 intercept)
on Table 1's A20 channel, run by validation.run on the GPU in FP64, against
the oracle's run with the same parameters: 100 steps of development, then
200 steps sampled every 20.  The sampled mean profile agrees to FP64
round-off of 300 steps (|d<u_x>| <= 1e-9 u_tau), and so do the metrics
computed from it.  Both wall pictures: halfway walls with WFB, wall nodes
with bounce-back (the paper's comparison path), and wall nodes with WFB whose
stress follows the first layer's velocity of the same step."""
import numpy as np
import pytest

from gpu_common import oracle_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_04352_amd as P
    return P


@pytest.mark.parametrize("bc,wall_nodes", (("wfb", 0), ("bb", 1), ("wfb", 2)))
def test_a20_statistics_and_metrics_match_oracle(P, orc, bc, wall_nodes):
    from paper_2009_04352_amd import validation as V
    from paper_2009_04352_amd import workloads as W
    print("validation A20 %s wall_nodes=%s" % (bc, wall_nodes), flush=True)
    m = V.run("A20", store="f64", bc=bc, collision="bgk", van_driest=0.0, develop=100, sample=200, stats_every=20,
              report_every=100, pdf_bins=8, wall_nodes=wall_nodes)
    assert m["status"] == 0 and m["sampled_steps"] == 10
    p = W.params("A20")
    nx, ny, nz = p["grid"]
    if wall_nodes:
        ny -= 1
    assert m["grid"] == [nx, ny, nz]
    o = oracle_for(orc, (nx, ny, nz), p["tau0"], p["cs"], p["fx"], bc, stats_every=20, wall_nodes=wall_nodes)
    o.init_spalding(p["u_tau"], p["noise"], p["seed"])
    assert o.step(100) == 0
    o.stats_reset()
    assert o.step(200) == 0
    sums, ns = o.stats_sums()
    assert ns == 10
    mean = sums[:, 0] / sums[:, 7]
    got = np.array(m["mean_ux"])
    assert np.abs(got - mean).max() <= 1e-9 * p["u_tau"], np.abs(got - mean).max() / p["u_tau"]
    want = V.profile_metrics(mean, p["u_tau"], p["nu0"])
    for k in ("eps_buffer", "eps_log", "eps_all", "b"):
        if want[k] is None:
            assert m[k] is None
        else:
            assert abs(m[k] - want[k]) <= 1e-6 * max(1.0, abs(want[k])), (k, m[k], want[k])
    np.testing.assert_allclose(m["yplus"], want["yplus"], rtol=1e-14)
