"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Small grids span several tiles and a ragged tail (nx = 67 = 64 + 3); every
store format, every boundary, both AA parities.  Comparisons are element by
element on the same seeded inputs with the tolerances of gpu_common.
"""
import zlib

import numpy as np
import pytest

from gpu_common import STORES, MATH_EPS, one_step_tol, oracle_for, random_state, ref_rounding, ulp, weights

pytestmark = pytest.mark.gpu

BCS = ("bb", "wfb", "freeslip")
GRIDS = [(4, 4, 4), (67, 5, 3)]
# degenerate geometries: one cell per row (x-periodic onto itself), one
# spanwise plane, and the thinnest channel (every row a wall row)
DEGENERATE = [(1, 5, 3), (8, 4, 1), (67, 2, 3)]


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_04352_amd as P
    return P


def _pair(P, orc, grid, store, bc, tau=0.52, cs=0.1, fx=2e-6, tiles=None, graph_steps=None, y1=1.0,
          stats_every=0):
    nx, ny, nz = grid
    ch = P.Channel(nx, ny, nz, tau, cs=cs, fx=fx, store=store, bc=bc, tiles=tiles, graph_steps=graph_steps, y1=y1,
                   stats_every=stats_every)
    o = oracle_for(orc, grid, tau, cs, fx, bc, y1=y1, stats_every=stats_every)
    return ch, o


@pytest.mark.parametrize("grid", GRIDS + DEGENERATE)
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("store", STORES)
def test_one_and_two_steps(P, orc, store, bc, grid):
    """One step from a representable state: each h_a within one ulp of the store
    plus the arithmetic bound; the second step (even kernel) starts from the
    GPU's own state handed to the oracle."""
    print("parity: %s %s %s" % (store, bc, grid), flush=True)
    rng = np.random.default_rng(zlib.crc32(repr((store, bc, grid)).encode()))
    nx, ny, nz = grid
    h0 = random_state(orc, (nz, ny, nx), store, rng)
    w = weights(orc)
    ch, o = _pair(P, orc, grid, store, bc)
    ch.set_state(h0)
    o.set_state(h0 + w)
    ch.step(1)
    o.step(1)
    assert ch.sync()[0] == 0
    got, want = ch.get_state(), o.state() - w
    assert np.all(np.abs(got - want) <= one_step_tol(store, want, w)), np.abs(got - want).max()
    # even kernel: continue the oracle from the GPU's rounded state
    o.set_state(got + w)
    ch.step(1)
    o.step(1)
    got, want = ch.get_state(), o.state() - w
    assert np.all(np.abs(got - want) <= one_step_tol(store, want, w)), np.abs(got - want).max()


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("store", STORES)
def test_observables_both_parities(P, orc, store, bc):
    """Moments and wall records of the current state agree with the oracle after
    an even and after an odd number of steps (both AA layouts)."""
    grid = (67, 5, 3)
    rng = np.random.default_rng(17)
    nx, ny, nz = grid
    w = weights(orc)
    ch, o = _pair(P, orc, grid, store, bc)
    ch.set_state(random_state(orc, (nz, ny, nx), store, rng))
    for k in range(3):
        o.set_state(ch.get_state() + w)
        mg, mo = ch.moments(), o.observe()
        tol = 8 * MATH_EPS[store]
        for a, b in zip(mg, mo):
            np.testing.assert_allclose(a, b, rtol=0, atol=tol)
        # wall records: the direction of tau follows the FP32 (or FP64) velocity
        # sums, so components are compared against the magnitude of the record
        wg, wo = ch.wall_shear(), o.wall()
        for a, b in zip(wg, wo):
            scale = np.abs(b).max() + 1e-300
            np.testing.assert_allclose(a, b, rtol=0, atol=(1e-5 if store != "f64" else 1e-12) * scale)
        cells = np.array([0, 1, nx - 1, nx, nx * ny - 1, nx * ny * nz - 1, 5 * nx + 3])
        mc = ch.moments_cells(cells)
        flat = [m.reshape(-1) for m in mg]
        np.testing.assert_array_equal(mc, np.stack([f[cells] for f in flat], axis=1))
        ch.step(1)


@pytest.mark.parametrize("bc", ("bb", "wfb"))
def test_fp64_c1_200_steps(P, orc, bc):
    """The 32x16x16 Re_tau 640 channel from its Spalding initial state, 200
    steps in FP64: max |du| / u_tau <= 1e-9 against the oracle, for the low-Mach
    relaxation time and for the named tau = 0.51."""
    from paper_2009_04352_amd import workloads as W
    for named in (False, True):
        p = W.params("c1", named_tau=named)
        ch, o = _pair(P, orc, p["grid"], "f64", bc, tau=p["tau0"], cs=p["cs"], fx=p["fx"])
        ch.init_spalding(p["u_tau"], p["noise"], p["seed"])
        o.init_spalding(p["u_tau"], p["noise"], p["seed"])
        ch.step(200)
        assert o.step(200) == 0
        assert ch.sync()[0] == 0
        mg, mo = ch.moments(), o.observe()
        assert np.abs(mg[0] - mo[0]).max() <= 1e-12
        du = max(np.abs(a - b).max() for a, b in zip(mg[1:], mo[1:]))
        assert du / p["u_tau"] <= 1e-9, du / p["u_tau"]


@pytest.mark.parametrize("store", STORES)
def test_initial_state(P, orc, store):
    """Spalding profile with splitmix64 noise, rounded once to the store."""
    from paper_2009_04352_amd import workloads as W
    p = W.params("c1")
    ch, o = _pair(P, orc, p["grid"], store, "wfb", tau=p["tau0"], fx=p["fx"])
    ch.init_spalding(p["u_tau"], 0.05, 12345)
    o.init_spalding(p["u_tau"], 0.05, 12345)
    w = weights(orc)
    got, want = ch.get_state(), o.state() - w
    # one rounding to the store plus the reference's own rounding of f - w
    tol = ulp(store, want) + ref_rounding(w, want)
    assert np.all(np.abs(got - want) <= tol)


def test_device_newton_matches_spalding(P, orc):
    """The kernel's FP64 Newton solve (started from an FP32 estimate, where the
    oracle starts from the viscous guess): Spalding residual <= 1e-10 and u_tau
    equal to the oracle's to 1e-13 relative; few FP64 steps at any R."""
    U = np.geomspace(1e-7, 0.2, 200)
    for y1, nu in ((1.0, 2.04e-5), (1.0, 1e-3), (0.5, 1e-4)):
        ut, it = P.device_wall_utau(U, y1, nu)
        assert np.all(ut > 0) and np.all(it >= 1) and np.all(it <= 6)
        for Ui, ui in zip(U, ut):
            yp, up = y1 * ui / nu, Ui / ui
            assert abs(orc.spalding_yplus(up) - yp) <= 1e-10 * yp
            ref, _ = orc.wall_utau(Ui, y1, nu)
            assert abs(ui - ref) <= 1e-13 * ref
    ut, it = P.device_wall_utau(np.array([0.0, 1.0]), 1.0, 1e-5)
    assert ut[0] == 0.0 and it[0] == 0
    assert ut[1] > 0.0 and it[1] <= 6        # R = 1e5: the FP32 start leaves a few FP64 steps
    ut, it = P.device_wall_utau(np.array([0.0, 1e-2]), 1.0, 1e-5, maxit=1)
    assert ut[1] == -1.0 and it[1] == 1      # beyond the cap: reported, not returned


@pytest.mark.parametrize("bc", BCS)
def test_mass_and_momentum_budget(P, orc, bc):
    """Mass conserved to 1e-12 over 200 FP64 steps; each step's x-momentum
    change equals N Fx plus the wall force of the next state."""
    from paper_2009_04352_amd import workloads as W
    p = W.params("c1", named_tau=True)
    ch, _ = _pair(P, orc, p["grid"], "f64", bc, tau=p["tau0"], fx=p["fx"])
    ch.init_spalding(p["u_tau"], 0.05, 3)
    n = np.prod(p["grid"])

    def totals():
        rho, ux, _, _ = ch.moments()
        return rho.sum(), (rho * ux).sum()

    m0, j0 = totals()
    for _ in range(5):
        ch.step(1)
        m1, j1 = totals()
        tx = ch.wall_shear()[0]
        assert abs((j1 - j0) - (n * p["fx"] + tx.sum())) <= 1e-9 * n * p["fx"] + 1e-14 * abs(j0)
        j0 = j1
    ch.step(195)
    m1, _ = totals()
    assert abs(m1 - m0) <= 1e-12 * m0


def test_poiseuille_on_gpu(P):
    """BGK + Guo + halfway bounce-back on a 1 x 32 x 1 channel (Cs = 0): the
    converged profile is the parabola plus the exact wall slip."""
    tau, ny, F = 0.8, 32, 1e-6
    ch = P.Channel(1, ny, 1, tau, cs=0.0, fx=F, store="f64", bc="bb")
    nu, s = (tau - 0.5) / 3.0, tau - 0.5
    y = np.arange(ny) + 0.5
    exact = F / (2 * nu) * y * (ny - y) + F * (16 * s * s - 3) / (8 * s)
    ch.init_spalding(0.0, 0.0, 0)
    ch.step(30000)
    _, ux, _, _ = ch.moments()
    u = ux[0, :, 0]
    assert np.abs(u - exact).max() <= 1e-10 * exact.max()


def test_freeslip_fixed_point_on_gpu(P, orc):
    e, w, _, _ = orc.tables()
    nx, ny, nz = 70, 5, 4
    f1 = orc.feq(1.0, np.array([0.04, 0.0, -0.03])) - w
    h0 = np.broadcast_to(f1[:, None, None, None], (19, nz, ny, nx)).copy()
    ch = P.Channel(nx, ny, nz, 0.53, cs=0.1, fx=0.0, store="f64", bc="freeslip")
    ch.set_state(h0)
    ch.step(25)
    assert np.abs(ch.get_state() - h0).max() <= 1e-15
    ch.set_boundary("bb")
    ch.step(5)
    assert np.abs(ch.get_state() - h0).max() > 1e-4


def test_wfb_laminar_force_balance_on_gpu(P):
    ny, F, tau = 16, 1e-6, 0.8
    ch = P.Channel(1, ny, 1, tau, cs=0.0, fx=F, store="f64", bc="wfb")
    ch.init_spalding(0.0, 0.0, 0)
    ch.step(20000)
    tx, tz, ut, U = ch.wall_shear()
    rho = ch.moments()[0]
    assert abs(tx.mean() + F * ny / 2) <= 1e-10 * F * ny / 2
    assert abs(rho[0, 0, 0] * ut[0, 0, 0] ** 2 - F * ny / 2) <= 1e-10 * F * ny / 2


def test_statistics_match_oracle(P, orc):
    """FP64 plane sums of the sampled velocities, every second step."""
    grid = (67, 6, 5)
    rng = np.random.default_rng(4)
    w = weights(orc)
    ch, o = _pair(P, orc, grid, "f64", "wfb", stats_every=2)
    h0 = random_state(orc, grid[::-1], "f64", rng)
    ch.set_state(h0)
    o.set_state(h0 + w)
    ch.step(7)
    o.step(7)
    sg, ng = ch.stats_sums()
    so, no = o.stats_sums()
    assert ng == no == 3
    # sums of signed velocities cancel: compare against the summed magnitudes
    assert np.all(np.abs(sg - so) <= 1e-12 * np.abs(so) + 1e-14 * so[:, 7:8]), np.abs(sg - so).max()
    st, _ = ch.stats()
    np.testing.assert_allclose(st[:, 0], so[:, 0] / so[:, 7], rtol=1e-12, atol=1e-17)
    ch.stats_reset()
    assert ch.stats_sums()[1] == 0 and np.all(ch.stats_sums()[0] == 0)


def test_statistics_with_many_rows_per_block(P, orc):
    """Short rows packed many to a block (16 cells, 4 per thread: 32 rows per
    128-thread block) still give every layer its plane sums."""
    grid = (16, 40, 3)
    rng = np.random.default_rng(12)
    w = weights(orc)
    ch, o = _pair(P, orc, grid, "f16", "wfb", stats_every=1, tiles=(128, 128, 4))
    h0 = random_state(orc, grid[::-1], "f16", rng)
    ch.set_state(h0)
    o.set_state(h0 + w)
    ch.step(2)
    o.step(2)
    sg, ng = ch.stats_sums()
    so, no = o.stats_sums()
    assert ng == no == 2
    np.testing.assert_array_equal(sg[:, 7], so[:, 7])
    # the second sample sees the state rounded once to FP16: per cell at most 19
    # half-ulps of FP16 at |h| < 0.03 (7.6e-6 each) in each velocity component
    assert np.all(np.abs(sg[:, :7] - so[:, :7]) <= 2e-4 * so[:, 7:8]), np.abs(sg - so).max()


def test_boundary_switch_after_odd_step(P, orc):
    """Switching the boundary between an odd and an even step re-reflects the
    pending wall populations: the result equals the oracle, which reflects at
    gather time with the new rule."""
    grid = (66, 4, 3)
    rng = np.random.default_rng(8)
    w = weights(orc)
    for first, second in (("wfb", "bb"), ("bb", "wfb"), ("freeslip", "wfb")):
        ch, o = _pair(P, orc, grid, "f64", first)
        h0 = random_state(orc, grid[::-1], "f64", rng)
        ch.set_state(h0)
        o.set_state(h0 + w)
        ch.step(1)
        o.step(1)
        ch.set_boundary(second)
        o.set_bc({"bb": orc.BB, "wfb": orc.WFB, "freeslip": orc.FREESLIP}[second])
        ch.step(2)
        o.step(2)
        np.testing.assert_allclose(ch.get_state(), o.state() - w, rtol=0, atol=2e-15)


# (boundary, wall placement): halfway walls, wall nodes, and wall nodes with
# the same step's stress (which only differs from the previous step's with WFB)
REST_CASES = [(bc, m) for bc in BCS for m in (0, 1)] + [("wfb", 2)]


@pytest.mark.parametrize("bc,wall_nodes", REST_CASES)
@pytest.mark.parametrize("store", STORES)
def test_fluid_at_rest_stays_at_rest(P, store, bc, wall_nodes):
    """The degenerate flow: no force and f = f_eq(1, 0) everywhere.  Every
    population stays exactly at its weight (h = 0 in every format), the wall
    function sees U = 0 and returns u_tau = 0 without a Newton step, and every
    wall stress is exactly zero, for each boundary and wall placement."""
    from paper_2009_04352_amd import _lib as L
    nx, ny, nz = 24, 5, 3
    ch = P.Channel(nx, ny, nz, 0.52, cs=0.1, fx=0.0, store=store, bc=bc, wall_nodes=wall_nodes)
    # a cap of one iteration: any solve that needed a step would be reported
    ch.set_param(L.LBM_P_NEWTON_MAXIT, 1)
    ch.init_moments(np.ones((nz, ny, nx)), np.zeros((3, nz, ny, nx)))
    ch.step(7)
    assert ch.sync()[0] == 0
    assert not np.any(ch.get_state())
    for a in ch.wall_shear()[:3]:
        assert not np.any(a)
    if wall_nodes:
        fw, rec = ch.wall_nodes()
        assert not np.any(fw) and not np.any(rec[..., 1:])
