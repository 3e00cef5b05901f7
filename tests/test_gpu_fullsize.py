"""Parity at the benchmark's full sizes (512 x 128 x 256 channel, 16.8M cells;
2048 x 512 x 1024 channel, 1.07G cells) in the launch configuration the
benchmark times: sampled cells after one step
against the oracle evaluated cell by cell from the analytic initial state, and
conservation properties that hold at any size."""
import numpy as np
import pytest

from gpu_common import MATH_EPS, one_step_tol, ref_rounding, ulp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_04352_amd as P
    return P


def _channel(P, store, named=False, workload="c3", collision="bgk", van_driest=0.0, grid=None, tune=False):
    from paper_2009_04352_amd import workloads as W
    p = W.params(workload, named_tau=named)
    if grid is not None:
        p = dict(p, grid=grid)
    ch = P.Channel(*p["grid"], p["tau0"], cs=p["cs"], fx=p["fx"], store=store, bc="wfb",
                   tiles=W.launch_tiles(workload, store, collision), collision=collision, van_driest=van_driest)
    if tune:   # as the benchmark does: the tuner searches from the table before the state is set
        print("tuned launch:", ch.autotune(steps=4), flush=True)
    ch.init_spalding(p["u_tau"], p["noise"], p["seed"])
    return ch, p


def _release(ch):
    import torch
    ch.close()
    del ch
    torch.cuda.empty_cache()


# the benchmark's workloads and stores: the 2048 x 512 x 1024 channel (1.07 G
# cells) in all four formats, the 512 x 128 x 256 channel in all four formats
# and at its named relaxation time tau = 0.503 (FP64 and FP16), and one GPU's
# 256 x 512 x 1024 x-slab of the large channel (FP64, FP16)
FULL = [("c5", "f64", "bgk", False), ("c5", "f32", "bgk", False), ("c5", "f16", "bgk", False),
        ("c5", "bf16", "bgk", False),
        ("c3", "f64", "bgk", False), ("c3", "f32", "bgk", False), ("c3", "f16", "bgk", False),
        ("c3", "bf16", "bgk", False), ("c3", "f64", "bgk", True), ("c3", "f16", "bgk", True),
        ("c5s", "f64", "bgk", False), ("c5s", "f16", "bgk", False)]


# the MRT line of the benchmark (--collision mrt --van-driest 26) on the
# 512 x 128 x 256 channel, and on the 2048 x 512 x 1024 channel (where the
# 2-byte odd step walks rows at 2 cells per thread)
FULL_MRT = [("c3", "f64", "mrt", False), ("c3", "f32", "mrt", False), ("c3", "f16", "mrt", False),
            ("c3", "bf16", "mrt", False), ("c5", "f64", "mrt", False), ("c5", "f16", "mrt", False),
            ("c5", "bf16", "mrt", False)]


@pytest.mark.parametrize("workload,store,collision,named", FULL + FULL_MRT)
def test_two_steps_sampled(P, orc, workload, store, collision, named):
    """Step 1 (odd kernel) at sampled cells against the oracle evaluated cell by
    cell from the analytic initial state; tolerance: the initial rounding to
    the store (half an ulp of each input population, carried through one
    collision with relaxation factor below 2 into at most 19 terms) plus one
    ulp of the output and the arithmetic bound.  Step 2 (even kernel, in its
    full-size launch shape) at the same cells against the oracle's step from
    the GPU's own step-1 state of the cells around them, with the one-step
    tolerance (one ulp of the store at the result, the arithmetic bound and the
    oracle's own rounding)."""
    _two_steps_sampled(P, orc, workload, store, collision, named)


@pytest.mark.parametrize("store", ("f64", "f32", "f16", "bf16"))
def test_two_steps_sampled_in_tuned_shapes(P, orc, store):
    """The two sampled steps on the 2048 x 512 x 1024 channel in the shapes the
    benchmark's autotuner picks on this device (block sizes, cells per thread,
    rows per brick, launch order, odd-step mode)."""
    _two_steps_sampled(P, orc, "c5", store, "bgk", False, tune=True)


# The largest grid the library takes is just below 2^31 cells: 2048 x 1023 x
# 1024 (99.9 % of the limit; the odd row count leaves a last brick of 7 rows)
# in the large channel's parameters and launch shapes, in the formats whose
# populations fit in one GPU's memory at that size (FP16 81.5 GB, FP32
# 163 GB; FP64 would need 326 GB).
LARGEST = (2048, 1023, 1024)


@pytest.mark.parametrize("store", ("f16", "f32"))
def test_largest_grid_two_steps_sampled(P, orc, store):
    """The two sampled steps of the test above on the largest accepted grid."""
    assert np.prod(LARGEST) < 2 ** 31 and np.prod(LARGEST) > 0.999 * 2 ** 31
    _two_steps_sampled(P, orc, "c5", store, "bgk", False, grid=LARGEST)


def _two_steps_sampled(P, orc, workload, store, collision, named, grid=None, tune=False):
    from paper_2009_04352_amd import workloads as W
    print("full-size sampled steps: %s %s %s named=%s grid=%s tuned=%s" % (workload, store, collision, named, grid,
                                                                         tune), flush=True)
    vd = 26.0 if collision == "mrt" else 0.0
    ch, p = _channel(P, store, named=named, workload=workload, collision=collision, van_driest=vd, grid=grid,
                     tune=tune)
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
    # step 2: the even kernel, from the GPU's step-1 state around the samples
    tab = orc.neighbourhood(p["grid"], cells)
    h1 = ch.get_state_cells(tab)
    ch.step(1)
    want2, _ = orc.step_cells_table(op, tab, h1 + w, cells)
    want2 -= w
    got2 = ch.get_state_cells(cells)
    assert np.all(np.abs(got2 - want2) <= one_step_tol(store, want2, w)), np.abs(got2 - want2).max()
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


@pytest.mark.parametrize("bc,mode", (("wfb", 1), ("wfb", 2), ("bb", 1)))
def test_c3_fp64_wall_nodes_budget(P, orc, bc, mode):
    """Wall nodes (Sec. 2.1-2.2) at full size in the benchmark's FP64 launch
    shape: per step the x-momentum of fluid plus wall nodes changes by N Fx
    plus the stress of the step's wall-node collisions (WFB: from the record
    before the step, or with the same step's velocity from the one the step
    computed; bounce-back: the momentum exchange of the populations waiting
    at the nodes), and their mass is conserved."""
    from paper_2009_04352_amd import workloads as W
    print("full-size wall nodes: c3 f64 %s mode %d" % (bc, mode), flush=True)
    p = W.params("c3")
    nx, ny, nz = p["grid"]
    ch = P.Channel(nx, ny, nz, p["tau0"], cs=p["cs"], fx=p["fx"], store="f64", bc=bc,
                   tiles=W.launch_tiles("c3", "f64"), wall_nodes=mode)
    ch.init_spalding(p["u_tau"], p["noise"], p["seed"])
    ex = orc.tables()[0][:, 0].astype(np.float64)
    ex_in = np.array([[ex[a] for a in orc.IN_W[k]] for k in (0, 1)])

    def totals():
        # h = f - w: sum_a w_a and sum_a e_ax w_a are constants (zero for x-momentum)
        h = ch.get_state().reshape(19, -1)
        fw, _ = ch.wall_nodes()
        fw = fw.reshape(2, 5, -1)
        m = h.sum() + fw.sum()
        px = float(ex @ h.sum(axis=1)) + float((ex_in * fw.sum(axis=2)).sum())
        return m, px, np.abs(h).sum()

    n = nx * ny * nz
    m0, _, _ = totals()
    for _ in range(2):
        _, p0, habs = totals()
        taux = ch.wall_shear()[0]
        ch.step(1)
        if mode == 2 and bc == "wfb":
            taux = ch.wall_shear()[0]   # the stress of the step's own record
        _, p1, _ = totals()
        want = n * p["fx"] + taux.sum()
        # pairwise sums over 3e8 terms: a few ulp of the summed magnitudes
        assert abs((p1 - p0) - want) <= 1e-9 * abs(want) + 1e-14 * habs, ((p1 - p0), want)
    ch.step(20)
    m1, _, habs = totals()
    assert abs(m1 - m0) <= 1e-14 * habs, (m1 - m0)
    assert ch.sync()[0] == 0
    _release(ch)
