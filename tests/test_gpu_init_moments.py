"""lbm_init_moments: the post-collision state f_eq(rho, u) of Eq. 1 computed on
the device from host moments, against the oracle's equilibrium, on a grid
with ragged tiles, for every store format; bad moments are refused."""
import numpy as np
import pytest

from gpu_common import STORES, one_step_tol, round_to

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_04352_amd as P
    return P


def _moments(shape, seed=11):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    rho = 1.0 + 0.05 * (2.0 * rng.random(shape) - 1.0)
    u = 0.05 * rng.standard_normal((3,) + shape)
    return rho, u


@pytest.mark.parametrize("store", STORES)
def test_init_moments_is_the_equilibrium(P, orc, store):
    nx, ny, nz = 40, 12, 6
    rho, u = _moments((nz, ny, nx))
    ch = P.Channel(nx, ny, nz, 0.55, fx=1e-6, store=store, bc="wfb")
    ch.init_moments(rho, u)
    got = ch.get_state().reshape(19, nz, ny, nx)
    _, w, _, _ = orc.tables()
    want = np.empty_like(got)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                want[:, z, y, x] = orc.feq(rho[z, y, x], u[:, z, y, x]) - w
    wb = w[:, None, None, None]
    assert np.all(np.abs(got - want) <= one_step_tol(store, want, wb)), np.abs(got - want).max()
    # what the device stored is a value of the store format
    assert np.array_equal(got, round_to(store, got))
    assert ch.steps == 0
    ch.close()


def test_init_moments_then_steps_like_set_state(P):
    nx, ny, nz = 64, 16, 8
    rho, u = _moments((nz, ny, nx), seed=5)
    a = P.Channel(nx, ny, nz, 0.52, fx=1e-6, store="f16", bc="wfb")
    a.init_moments(rho, u)
    h0 = a.get_state()
    b = P.Channel(nx, ny, nz, 0.52, fx=1e-6, store="f16", bc="wfb")
    b.set_state(h0, 0)
    a.step(5)
    b.step(5)
    assert np.array_equal(a.get_state(), b.get_state())
    a.close()
    b.close()


def test_init_moments_refuses_bad_moments(P):
    nx, ny, nz = 16, 8, 4
    ch = P.Channel(nx, ny, nz, 0.55, store="f32", bc="wfb")
    rho, u = _moments((nz, ny, nx))
    ch.init_moments(rho, u)
    before = ch.get_state()
    bad = rho.copy()
    bad[1, 2, 3] = 0.0
    with pytest.raises(P.LbmError):
        ch.init_moments(bad, u)
    u2 = u.copy()
    u2[0, 0, 0, 0] = np.nan
    with pytest.raises(P.LbmError):
        ch.init_moments(rho, u2)
    with pytest.raises(ValueError):
        ch.init_moments(rho[:, :, :-1], u)
    ch.init_moments(rho, u)
    assert np.array_equal(ch.get_state(), before)
    ch.close()
