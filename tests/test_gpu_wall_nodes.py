"""GPU parity of the wall-node picture (LBM_P_WALL_NODES = 1: the wall grid of
Sec. 2.1-2.2 as a lattice node one spacing outside the first fluid layer,
Eq. 3, 4 and 14 applied there, one step of lag and twice the tangential
shift of the halfway walls) against the FP64 oracle's wall-node mode.

One and two steps from a representable state, every store format, every
boundary, grids with a ragged tail and several cells per thread: the fluid
populations and the wall nodes' outputs within the one-step tolerance of
gpu_common (one ulp of the store at the result, the arithmetic bound and the
oracle's own rounding), the first-layer records (density, velocity) within
the observables' bound; the oracle continues from the GPU's rounded state,
wall nodes included.  200 FP64 steps of the 32x16x16 channel from its
Spalding state: max |du| / u_tau <= 1e-9.  Mode 2 (the stress from the
first layer's velocity of the same step) runs the same checks with WFB, the
only boundary where the two modes differ.
"""
import zlib

import numpy as np
import pytest

from gpu_common import MATH_EPS, STORES, one_step_tol, oracle_for, random_state, weights

pytestmark = pytest.mark.gpu

BCS = ("bb", "wfb", "freeslip")
# (boundary, mode): the stress timing of mode 2 only matters for WFB
BC_MODES = [("bb", 1), ("wfb", 1), ("freeslip", 1), ("wfb", 2)]
GRIDS = [(4, 4, 4), (67, 5, 3), (64, 6, 3)]
# degenerate geometries: one cell per row with a single wall-adjacent row
# pair, and one spanwise plane with every row next to a wall node
DEGENERATE = [(1, 3, 2), (8, 2, 1)]


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_04352_amd as P
    return P


def _pair(P, orc, grid, store, bc, tau=0.52, cs=0.1, fx=2e-6, mode=1, **kw):
    nx, ny, nz = grid
    ch = P.Channel(nx, ny, nz, tau, cs=cs, fx=fx, store=store, bc=bc, wall_nodes=mode, **kw)
    o = oracle_for(orc, grid, tau, cs, fx, bc, wall_nodes=mode)
    return ch, o


def _w_in(orc):
    """Weights of the wall nodes' output directions, [2, 5, 1, 1]."""
    w = orc.tables()[1]
    return np.array([[w[a] for a in orc.IN_W[k]] for k in (0, 1)])[:, :, None, None]


def _check(ch, o, orc, store, w, w_in):
    """Compares the state and the wall nodes, then continues the oracle from the
    GPU's rounded state (wall nodes included) and compares the wall records:
    the stress of the next wall-node collision (WFB, from the first-layer
    record) or the momentum exchange of the waiting populations (bounce-back)."""
    got, want = ch.get_state(), o.state() - w
    assert np.all(np.abs(got - want) <= one_step_tol(store, want, w)), ("fluid", np.abs(got - want).max())
    fg, rg = ch.wall_nodes()
    fo, uo = o.wall_nodes()
    fo = fo - w_in
    assert np.all(np.abs(fg - fo) <= one_step_tol(store, fo, w_in)), ("wall nodes", np.abs(fg - fo).max())
    tol = 8 * MATH_EPS[store]
    np.testing.assert_allclose(rg[..., :3], uo, rtol=0, atol=tol)
    o.set_state(got + w)
    o.set_wall_nodes(fg + w_in, rg[..., :3])
    wg, wo = ch.wall_shear(), o.wall()
    for a, b in zip(wg, wo):
        scale = np.abs(b).max() + 1e-300
        np.testing.assert_allclose(a, b, rtol=0, atol=(1e-5 if store != "f64" else 1e-12) * scale)


@pytest.mark.parametrize("grid", GRIDS + DEGENERATE)
@pytest.mark.parametrize("bc,mode", BC_MODES)
@pytest.mark.parametrize("store", STORES)
def test_wall_nodes_one_and_two_steps(P, orc, store, bc, mode, grid):
    print("wall nodes: %s %s mode %d %s" % (store, bc, mode, grid), flush=True)
    rng = np.random.default_rng(zlib.crc32(repr(("nodes", store, bc, grid) + ((mode,) if mode != 1 else ())).encode()))
    nx, ny, nz = grid
    h0 = random_state(orc, (nz, ny, nx), store, rng)
    w, w_in = weights(orc), _w_in(orc)
    ch, o = _pair(P, orc, grid, store, bc, mode=mode)
    ch.set_state(h0)
    o.set_state(h0 + w)
    _check(ch, o, orc, store, w, w_in)          # the wall nodes' start
    for _ in range(2):                          # the odd, then the even kernel
        ch.step(1)
        assert o.step(1) == 0
        assert ch.sync()[0] == 0
        _check(ch, o, orc, store, w, w_in)


@pytest.mark.parametrize("bc,mode", (("wfb", 1), ("bb", 1), ("wfb", 2)))
def test_wall_nodes_fp64_200_steps(P, orc, bc, mode):
    """The 32x15x16 channel (the wall nodes add a spacing: 2D = 16) from its
    Spalding state, 200 FP64 steps against the oracle."""
    from paper_2009_04352_amd import workloads as W
    p = W.params("c1")
    nx, _, nz = p["grid"]
    grid = (nx, 15, nz)
    ch, o = _pair(P, orc, grid, "f64", bc, tau=p["tau0"], cs=p["cs"], fx=p["fx"], mode=mode)
    ch.init_spalding(p["u_tau"], p["noise"], p["seed"])
    o.init_spalding(p["u_tau"], p["noise"], p["seed"])
    ch.step(200)
    assert o.step(200) == 0
    assert ch.sync()[0] == 0
    mg, mo = ch.moments(), o.observe()
    assert np.abs(mg[0] - mo[0]).max() <= 1e-12
    du = max(np.abs(a - b).max() for a, b in zip(mg[1:], mo[1:]))
    assert du / p["u_tau"] <= 1e-9, du / p["u_tau"]
    fg, _ = ch.wall_nodes()
    fo, _ = o.wall_nodes()
    assert np.abs(fg - (fo - _w_in(orc))).max() <= 1e-12


@pytest.mark.parametrize("store,mode", (("f64", 1), ("f16", 1), ("f16", 2)))
def test_wall_nodes_graph_equals_eager(P, orc, store, mode):
    """Captured graph chunks and eager launches give the same bits (the wall-node
    rings alternate with the kernel parity, not with the step count)."""
    from paper_2009_04352_amd import workloads as W
    p = W.params("c1")
    nx, ny, nz = 64, 15, 8
    outs = []
    for gs in (0, 16):
        ch = P.Channel(nx, ny, nz, p["tau0"], cs=p["cs"], fx=p["fx"], store=store, bc="wfb", wall_nodes=mode,
                       graph_steps=gs)
        ch.init_spalding(p["u_tau"], p["noise"], p["seed"])
        ch.step(37)
        assert ch.sync()[0] == 0
        outs.append((ch.get_state(), ch.wall_nodes()))
        ch.close()
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    for a, b in zip(outs[0][1], outs[1][1]):
        np.testing.assert_array_equal(a, b)


def test_wall_nodes_statistics_and_parameters(P, orc):
    """Plane statistics with wall nodes match the oracle's; the wall placement
    is fixed once the state is initialised; the Appendix B mass check is not
    defined for wall nodes."""
    from paper_2009_04352_amd import _lib as L
    from paper_2009_04352_amd import workloads as W
    p = W.params("c1")
    grid = (32, 15, 16)
    ch, o = _pair(P, orc, grid, "f64", "wfb", tau=p["tau0"], cs=p["cs"], fx=p["fx"], stats_every=1)
    o = oracle_for(orc, grid, p["tau0"], p["cs"], p["fx"], "wfb", stats_every=1, wall_nodes=True)
    ch.init_spalding(p["u_tau"], p["noise"], p["seed"])
    o.init_spalding(p["u_tau"], p["noise"], p["seed"])
    ch.step(20)
    assert o.step(20) == 0
    sg, ng = ch.stats_sums()
    so, no = o.stats_sums()
    assert ng == no == 20
    np.testing.assert_array_equal(sg[:, 7], so[:, 7])
    # sums of signed velocities cancel: the bound scales with the number of summed cells
    assert np.all(np.abs(sg - so) <= 1e-12 * np.abs(so) + 1e-14 * so[:, 7:8]), np.abs(sg - so).max()
    with pytest.raises(L.LbmError):
        ch.set_param(L.LBM_P_WALL_NODES, 0)
    with pytest.raises(L.LbmError):
        ch.wall_mass_change()
    assert ch.get_param(L.LBM_P_WALL_NODES) == 1.0
    assert ch.get_param(L.LBM_P_ODD_BY_ROWS) == 0.0
