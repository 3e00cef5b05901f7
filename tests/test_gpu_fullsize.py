"""Parity at the benchmark's full sizes (512 x 128 x 256 channel, 16.8M cells;
2048 x 512 x 1024 channel, 1.07G cells) in the launch configuration the
benchmark times: sampled cells after one step
against the oracle evaluated cell by cell from the analytic initial state, and
conservation properties that hold at any size."""
import numpy as np
import pytest

from gpu_common import MATH_EPS, ref_rounding, ulp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_04352_amd as P
    return P


def _channel(P, store, named=False, workload="c3", collision="bgk", van_driest=0.0):
    from paper_2009_04352_amd import workloads as W
    p = W.params(workload, named_tau=named)
    ch = P.Channel(*p["grid"], p["tau0"], cs=p["cs"], fx=p["fx"], store=store, bc="wfb",
                   tiles=W.launch_tiles(workload, store, collision), collision=collision, van_driest=van_driest)
    ch.init_spalding(p["u_tau"], p["noise"], p["seed"])
    return ch, p


def _release(ch):
    import torch
    ch.close()
    del ch
    torch.cuda.empty_cache()


# the benchmark's workloads and stores: the 512 x 128 x 256 channel in all four
# formats, the 2048 x 512 x 1024 channel (1.07 G cells) in FP16 and FP32 and
# its FP64 reference
FULL = [("c3", "f64"), ("c3", "f32"), ("c3", "f16"), ("c3", "bf16"), ("c5", "f16"), ("c5", "f32"), ("c5", "f64")]


# the MRT line of the benchmark (--collision mrt --van-driest 26) on the
# 512 x 128 x 256 channel
FULL_MRT = [("c3", "f64", "mrt"), ("c3", "f32", "mrt"), ("c3", "f16", "mrt"), ("c3", "bf16", "mrt")]


@pytest.mark.parametrize("workload,store,collision", [f + ("bgk",) for f in FULL] + FULL_MRT)
def test_one_step_sampled(P, orc, workload, store, collision):
    """Tolerance: the initial rounding to the store (half an ulp of each input
    population, carried through one collision with relaxation factor below 2
    into at most 19 terms) plus one ulp of the output and the arithmetic bound."""
    from paper_2009_04352_amd import workloads as W
    print("full-size sampled step: %s %s %s" % (workload, store, collision), flush=True)
    vd = 26.0 if collision == "mrt" else 0.0
    ch, p = _channel(P, store, workload=workload, collision=collision, van_driest=vd)
    cells = W.sample_cells(p["grid"], 3000, seed=1)
    nx, ny, nz = p["grid"]
    op = orc.make_params(nx, ny, nz, p["tau0"], cs=p["cs"], fx=p["fx"], bc=orc.WFB,
                         collision=orc.MRT if collision == "mrt" else orc.BGK, vd_aplus=vd)
    w = orc.tables()[1][None, :]
    h_init = orc.init_cells(op, p["u_tau"], p["noise"], p["seed"], cells) - w
    ref_round = ref_rounding(w, h_init)   # the oracle's f - w in FP64
    got0 = ch.get_state_cells(cells)
    assert np.all(np.abs(got0 - h_init) <= ulp(store, h_init) + ref_round)
    ch.step(1)
    want, mom0 = orc.step1_cells(op, p["u_tau"], p["noise"], p["seed"], cells)
    want -= w
    got = ch.get_state_cells(cells)
    hmax = np.abs(h_init).max()
    tol = ulp(store, want) + 4.0 * ulp(store, hmax) + MATH_EPS[store] + 8.0 * np.spacing(1.0 / 3.0)
    assert np.all(np.abs(got - want) <= tol), np.abs(got - want).max()
    assert ch.sync()[0] == 0
    _release(ch)


def test_c3_fp64_conservation(P):
    """FP64 store at full size: mass conserved to 1e-12 and the x-momentum
    budget (N Fx plus the wall stress) per step."""
    ch, p = _channel(P, "f64")
    n = np.prod(p["grid"])

    def totals():
        rho, ux, _, _ = ch.moments()
        return rho.sum(dtype=np.float64), (rho * ux).sum(dtype=np.float64)

    m0, j0 = totals()
    for _ in range(2):
        ch.step(1)
        m1, j1 = totals()
        tx = ch.wall_shear()[0]
        want = n * p["fx"] + tx.sum()
        assert abs((j1 - j0) - want) <= 1e-8 * abs(want) + 1e-13 * abs(j0)
        j0 = j1
    ch.step(40)
    m1, _ = totals()
    assert abs(m1 - m0) <= 1e-12 * m0
    assert ch.sync()[0] == 0
    _release(ch)
