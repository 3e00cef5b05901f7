"""Pin of the oracle's cell-by-cell path from the analytic initial state
(orc_init_cells, orc_step1_cells), the reference of every full-size parity
case: on a small grid it must give exactly, bit for bit, what the array path
gives (orc_init_spalding, then one orc_step and orc_get_state; the initial
observables from orc_observe).  Both evaluate the same initial state
(f = f_eq(1, u0), Spalding profile and splitmix64 noise) and the same update
(gather with the wall rules of Eq. 3-4 and 14, WFB of Eq. 13-17, moments of
Eq. 2, Smagorinsky, BGK or MRT with the body force of Eq. 1), one from the
stored array and one from the closed form; a mistake in the analytic source
(a wrong cell index, a swapped component, a missing wrap) breaks the equality.

The grid is odd in every direction (12 x 7 x 5) so that index mistakes cannot
cancel by symmetry; every cell is checked, wall rows and periodic seams
included."""
import numpy as np
import pytest

GRID = (12, 7, 5)
CASES = [(coll, bc) for coll in ("bgk", "mrt") for bc in ("bb", "wfb", "freeslip")]


def _params(orc, coll, bc):
    nx, ny, nz = GRID
    b = {"bb": orc.BB, "wfb": orc.WFB, "freeslip": orc.FREESLIP}[bc]
    if coll == "mrt":
        return orc.make_params(nx, ny, nz, 0.5003, cs=0.1, fx=3e-6, bc=b, collision=orc.MRT, vd_aplus=26.0)
    return orc.make_params(nx, ny, nz, 0.5003, cs=0.1, fx=3e-6, bc=b)


@pytest.mark.parametrize("coll,bc", CASES)
def test_cell_path_equals_array_path(orc, coll, bc):
    nx, ny, nz = GRID
    u_tau, noise, seed = 0.004, 0.05, 11
    cells = np.arange(nx * ny * nz, dtype=np.int64)
    p = _params(orc, coll, bc)
    o = orc.Oracle(p)
    o.init_spalding(u_tau, noise, seed)
    f0 = o.state().reshape(19, -1).T              # [cell][a]
    rho0, ux0, uy0, uz0 = (m.reshape(-1) for m in o.observe())
    assert o.step(1) == orc.OK
    f1 = o.state().reshape(19, -1).T

    init = orc.init_cells(p, u_tau, noise, seed, cells)
    step1, mom = orc.step1_cells(p, u_tau, noise, seed, cells)
    np.testing.assert_array_equal(init, f0)
    np.testing.assert_array_equal(step1, f1)
    np.testing.assert_array_equal(mom, np.stack([rho0, ux0, uy0, uz0], axis=1))


def test_cell_path_on_a_subset_in_any_order(orc):
    """A shuffled subset with repeats gives the rows of the full evaluation."""
    nx, ny, nz = GRID
    p = _params(orc, "bgk", "wfb")
    all_cells = np.arange(nx * ny * nz, dtype=np.int64)
    full, mfull = orc.step1_cells(p, 0.004, 0.05, 3, all_cells)
    rng = np.random.default_rng(5)
    sub = rng.integers(0, nx * ny * nz, 50).astype(np.int64)
    part, mpart = orc.step1_cells(p, 0.004, 0.05, 3, sub)
    np.testing.assert_array_equal(part, full[sub])
    np.testing.assert_array_equal(mpart, mfull[sub])


@pytest.mark.parametrize("coll,bc", CASES)
def test_table_path_equals_array_path(orc, coll, bc):
    """One step from a table of post-collision populations (the source of the
    full-size second-step checks) equals the array path's step: from the whole
    state, and at a subset from its 3 x 3 x 3 neighbourhoods only."""
    nx, ny, nz = GRID
    p = _params(orc, coll, bc)
    o = orc.Oracle(p)
    o.init_spalding(0.004, 0.05, 21)
    assert o.step(1) == orc.OK
    f1 = o.state().reshape(19, -1).T.copy()        # [cell][a]
    rho1, ux1, uy1, uz1 = (m.reshape(-1) for m in o.observe())
    assert o.step(1) == orc.OK
    f2 = o.state().reshape(19, -1).T
    cells = np.arange(nx * ny * nz, dtype=np.int64)
    got, mom = orc.step_cells_table(p, cells, f1, cells)
    np.testing.assert_array_equal(got, f2)
    np.testing.assert_array_equal(mom, np.stack([rho1, ux1, uy1, uz1], axis=1))
    sub = np.array([0, 5, nx - 1, nx * ny - 1, nx * ny * nz - 1, 3 * nx + 7, nx * ny * 2 + nx * 3], dtype=np.int64)
    tab = orc.neighbourhood(GRID, sub)
    got, _ = orc.step_cells_table(p, tab, f1[tab], sub)
    np.testing.assert_array_equal(got, f2[sub])


def test_table_path_reports_a_missing_cell(orc):
    nx, ny, nz = GRID
    p = _params(orc, "bgk", "wfb")
    o = orc.Oracle(p)
    o.init_spalding(0.004, 0.05, 1)
    f0 = o.state().reshape(19, -1).T
    tab = orc.neighbourhood(GRID, [40])
    tab = tab[tab != 41]
    with pytest.raises(RuntimeError):
        orc.step_cells_table(p, tab, f0[tab], np.array([40], dtype=np.int64))
