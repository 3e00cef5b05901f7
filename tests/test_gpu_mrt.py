"""GPU parity of the MRT collision and the van Driest damping (the paper's
LES setting, Sec. 3.1) against the FP64 oracle, through the C ABI.

Same tolerances as the BGK path (gpu_common): the MRT correction adds sums of
at most 19 terms with coefficients below 30 divided by the row norms, well
inside the FP32 arithmetic bound for |h| < 0.05.
"""
import zlib

import numpy as np
import pytest

from gpu_common import STORES, one_step_tol, oracle_for, random_state, weights

pytestmark = pytest.mark.gpu

MRT = dict(collision="mrt", van_driest=26.0)


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_04352_amd as P
    return P


def _pair(P, orc, grid, store, bc, tau=0.52, cs=0.1, fx=2e-6, tiles=None, **kw):
    nx, ny, nz = grid
    ch = P.Channel(nx, ny, nz, tau, cs=cs, fx=fx, store=store, bc=bc, tiles=tiles, graph_steps=0, **kw)
    o = oracle_for(orc, grid, tau, cs, fx, bc, **kw)
    return ch, o


@pytest.mark.parametrize("bc", ("bb", "wfb", "freeslip"))
@pytest.mark.parametrize("store", STORES)
def test_mrt_one_and_two_steps(P, orc, store, bc):
    """One odd and one even step of MRT with van Driest damping from a
    representable state, every h_a within the one-step tolerance."""
    grid = (67, 5, 3)
    rng = np.random.default_rng(zlib.crc32(repr(("mrt", store, bc)).encode()))
    nx, ny, nz = grid
    h0 = random_state(orc, (nz, ny, nx), store, rng)
    w = weights(orc)
    ch, o = _pair(P, orc, grid, store, bc, **MRT)
    ch.set_state(h0)
    o.set_state(h0 + w)
    ch.step(1)
    o.step(1)
    assert ch.sync()[0] == 0
    got, want = ch.get_state(), o.state() - w
    assert np.all(np.abs(got - want) <= one_step_tol(store, want, w)), np.abs(got - want).max()
    o.set_state(got + w)
    ch.step(1)
    o.step(1)
    got, want = ch.get_state(), o.state() - w
    assert np.all(np.abs(got - want) <= one_step_tol(store, want, w)), np.abs(got - want).max()


@pytest.mark.parametrize("store", ("f64", "f32"))
def test_mrt_rates_reach_every_moment(P, orc, store):
    """Non-default rates for every moment class, odd and even step."""
    grid = (64, 6, 4)
    rates = dict(s_e=0.9, s_eps=1.7, s_q=1.05, s_pi=0.6, s_m=1.5)
    rng = np.random.default_rng(5)
    h0 = random_state(orc, grid[::-1], store, rng)
    w = weights(orc)
    ch, o = _pair(P, orc, grid, store, "wfb", collision="mrt", mrt_rates=rates)
    ch.set_state(h0)
    o.set_state(h0 + w)
    for _ in range(2):
        ch.step(1)
        o.step(1)
        got, want = ch.get_state(), o.state() - w
        assert np.all(np.abs(got - want) <= one_step_tol(store, want, w)), np.abs(got - want).max()
        o.set_state(got + w)


@pytest.mark.parametrize("bc", ("bb", "wfb"))
def test_mrt_fp64_c1_200_steps(P, orc, bc):
    """The 32x16x16 Re_tau 640 channel, MRT with van Driest damping, 200 FP64
    steps from its Spalding initial state: max |du| / u_tau <= 1e-9."""
    from paper_2009_04352_amd import workloads as W
    p = W.params("c1")
    ch, o = _pair(P, orc, p["grid"], "f64", bc, tau=p["tau0"], cs=p["cs"], fx=p["fx"], **MRT)
    ch.init_spalding(p["u_tau"], p["noise"], p["seed"])
    o.init_spalding(p["u_tau"], p["noise"], p["seed"])
    ch.step(200)
    assert o.step(200) == 0
    assert ch.sync()[0] == 0
    mg, mo = ch.moments(), o.observe()
    assert np.abs(mg[0] - mo[0]).max() <= 1e-12
    du = max(np.abs(a - b).max() for a, b in zip(mg[1:], mo[1:]))
    assert du / p["u_tau"] <= 1e-9, du / p["u_tau"]


def test_mrt_with_equal_rates_is_bgk(P, orc):
    """With Cs = 0 and every rate 1/tau the MRT kernels give the BGK kernels'
    result to FP64 rounding."""
    grid = (64, 6, 4)
    tau = 0.55
    r = 1.0 / tau
    rng = np.random.default_rng(8)
    h0 = random_state(orc, grid[::-1], "f64", rng)
    out = []
    for kw in (dict(), dict(collision="mrt", mrt_rates=dict(s_e=r, s_eps=r, s_q=r, s_pi=r, s_m=r))):
        ch = P.Channel(*grid, tau, cs=0.0, fx=1e-6, store="f64", bc="wfb", graph_steps=0, **kw)
        ch.set_state(h0)
        ch.step(3)
        out.append(ch.get_state())
    assert np.abs(out[0] - out[1]).max() <= 1e-16


@pytest.mark.parametrize("store,tiles", [("f16", (64, 64, 4)), ("f32", (128, 128, 2))])
def test_mrt_odd_step_by_rows_equals_blocks(P, orc, store, tiles):
    """The row-walking odd kernel and the block kernel agree bit for bit with MRT."""
    grid = (256, 6, 4)
    h0 = random_state(orc, grid[::-1], store, np.random.default_rng(9))
    out = []
    for mode in (0, 2):
        ch = P.Channel(*grid, 0.51, cs=0.1, fx=2e-6, store=store, bc="wfb", tiles=tiles, graph_steps=0, **MRT)
        ch.set_param(15, mode)
        ch.set_state(h0)
        ch.step(5)
        assert ch.sync()[0] == 0
        out.append(ch.get_state())
    assert np.array_equal(out[0], out[1])


def test_mrt_batch_equals_single(P):
    """A batch of MRT channels with van Driest damping equals each channel stepped alone."""
    specs = [dict(nx=64, ny=6, nz=3, tau=0.51, cs=0.1, fx=1e-6, bc="wfb"),
             dict(nx=32, ny=8, nz=4, tau=0.53, cs=0.1, fx=3e-6, bc="bb")]
    b = P.Batch(specs, store="f32", graph_steps=0, **MRT)
    b.init_spalding([1e-2, 2e-2], 0.05, seeds=[3, 4])
    b.step(6)
    assert b.sync()[0] == 0
    for i, s in enumerate(specs):
        ch = P.Channel(s["nx"], s["ny"], s["nz"], s["tau"], cs=s["cs"], fx=s["fx"], store="f32", bc=s["bc"],
                       graph_steps=0, **MRT)
        ch.init_spalding([1e-2, 2e-2][i], 0.05, 3 + i)
        ch.step(6)
        assert np.array_equal(b.instance(i).get_state(), ch.get_state()), i


def test_van_driest_table_follows_parameters(P, orc):
    """Changing A+ or Cs between steps takes effect on the next step (the
    per-row table is refreshed), graph replays included."""
    grid = (64, 8, 4)
    w = weights(orc)
    rng = np.random.default_rng(12)
    h0 = random_state(orc, grid[::-1], "f64", rng)
    ch = P.Channel(*grid, 0.51, cs=0.1, fx=2e-6, store="f64", bc="wfb", graph_steps=2, collision="mrt",
                   van_driest=26.0)
    ch.set_state(h0)
    ch.step(2)
    ch.set_param(24, 5.0)               # LBM_P_VD_APLUS
    ch.set_param(12, 0.15)              # LBM_P_CS
    ch.step(2)
    o = oracle_for(orc, grid, 0.51, 0.1, 2e-6, "wfb", collision="mrt", van_driest=26.0)
    o.set_state(h0 + w)
    o.step(2)
    o2 = oracle_for(orc, grid, 0.51, 0.15, 2e-6, "wfb", collision="mrt", van_driest=5.0)
    o2.set_state(o.state())
    o2.step(2)
    want = o2.state() - w
    got = ch.get_state()
    assert np.all(np.abs(got - want) <= 4 * one_step_tol("f64", want, w)), np.abs(got - want).max()
