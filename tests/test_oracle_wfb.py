"""Pins of the oracle's WFB boundary (Eq. 12-15, Eq. 14 on a tiny grid)."""
import numpy as np
import pytest

import golden_io


def _random_wall_state(orc, rng):
    rho = rng.uniform(0.95, 1.05)
    u = np.array([rng.uniform(-0.08, 0.08), rng.uniform(-0.01, 0.01), rng.uniform(-0.08, 0.08)])
    return orc.feq(rho, u) + rng.normal(0, 2e-4, 19)


@pytest.mark.parametrize("wall", [0, 1])
def test_wfb_single_cell_algebra(orc, wall):
    """Eq. 12a (pair sums kept), 12b/13 (pair differences shifted by tau),
    no mass change, momentum change (tau_x, 0, tau_z) (Eq. 9 with dt = dy = 1),
    and tau antiparallel to the wall velocity with |tau| = tau_w (Eq. 15)."""
    e, _, _, mir = orc.tables()
    rng = np.random.default_rng(11 + wall)
    p = orc.make_params(4, 4, 4, 0.5002, fx=1e-7)
    shifted, _ = golden_io.eq14()
    for _ in range(100):
        f = _random_wall_state(orc, rng)
        g, rec, st, it = orc.wfb_cell(p, wall, f)
        assert st == 0 and it >= 1
        taux, tauz, ut, U = rec
        tau = {"x": taux, "z": tauz}
        for a, _, s, c in shifted:
            a_w = a if wall == 0 else mir[a]
            assert abs((g[a_w] - f[a_w]) - s * 0.5 * tau[c]) <= 1e-17 + 1e-15 * abs(tau[c])
        changed = {a if wall == 0 else mir[a] for a, _, _, _ in shifted}
        for a in set(range(19)) - changed:
            assert g[a] == f[a]
        assert abs(g.sum() - f.sum()) <= 2 * np.spacing(f.sum())
        dj = e.T @ (g - f)
        np.testing.assert_allclose(dj, [taux, 0.0, tauz], rtol=0, atol=1e-16)
        # Eq. 15: tau opposite to the free-slip wall velocity
        jx = e[:, 0] @ f + 0.5 * p.fx
        jz = e[:, 2] @ f
        assert taux * jx + tauz * jz < 0
        assert abs(taux * jz - tauz * jx) <= 1e-12 * abs(taux * jx + tauz * jz)
        assert abs(np.hypot(taux, tauz) - f.sum() * ut * ut) <= 1e-14 * f.sum() * ut * ut
        assert abs(U - np.hypot(jx, jz) / f.sum()) <= 1e-13 * U


def test_wfb_zero_velocity_changes_nothing(orc):
    p = orc.make_params(4, 4, 4, 0.51, fx=0.0)
    f = orc.feq(1.0, np.zeros(3))
    g, rec, st, _ = orc.wfb_cell(p, 0, f)
    assert st == 0 and np.array_equal(g, f) and np.all(rec == 0.0)


def test_eq14_on_a_tiny_grid(orc):
    """Brute force on a 3x2x3 channel: the first step's pre-collision state of a
    bottom cell is Eq. 14a-b applied to its in-plane neighbours' post-collision
    populations; a top cell sees the mirror image; every other link streams."""
    e, w, opp, mir = orc.tables()
    nx, ny, nz = 3, 2, 3
    rng = np.random.default_rng(5)
    f0 = w[:, None, None, None] * (1 + rng.uniform(-0.1, 0.1, (19, nz, ny, nx)))
    p = orc.make_params(nx, ny, nz, 0.52, cs=0.0, fx=3e-6, bc=orc.WFB)
    o = orc.Oracle(p)
    o.set_state(f0)
    rho, ux, uy, uz = o.observe()
    taux, tauz, ut, U = o.wall()
    shifted, _ = golden_io.eq14()
    for z in range(nz):
        for x in range(nx):
            for y, wall in ((0, 0), (ny - 1, 1)):
                f = np.empty(19)
                for a in range(19):
                    sx, sy, sz = (x - e[a, 0]) % nx, y - e[a, 1], (z - e[a, 2]) % nz
                    if 0 <= sy < ny:
                        f[a] = f0[a, sz, sy, sx]
                    elif e[a, 0] == 0 and e[a, 2] == 0:
                        f[a] = f0[opp[a], z, y, x]
                    else:
                        f[a] = f0[mir[a], sz, y, sx]
                tau = {"x": taux[wall, z, x], "z": tauz[wall, z, x]}
                for a, b, s, c in shifted:
                    a_w, b_w = (a, b) if wall == 0 else (mir[a], mir[b])
                    dx, dz = -e[a_w, 0], -e[a_w, 2]
                    assert f[a_w] == f0[b_w, (z + dz) % nz, y, (x + dx) % nx]
                    f[a_w] += s * 0.5 * tau[c]
                r = f.sum()
                want_u = (e.T @ f + np.array([0.5 * p.fx, 0, 0])) / r
                assert abs(rho[z, y, x] - r) <= 1e-15
                np.testing.assert_allclose([ux[z, y, x], uy[z, y, x], uz[z, y, x]], want_u, atol=1e-16)


def test_freeslip_is_wfb_without_stress(orc):
    """With the stress switched off (free-slip) the same gather gives the
    mirror reflection only (Eq. 4 in 3-D form)."""
    nx, ny, nz = 4, 3, 2
    rng = np.random.default_rng(9)
    _, w, _, _ = orc.tables()
    f0 = w[:, None, None, None] * (1 + rng.uniform(-0.1, 0.1, (19, nz, ny, nx)))
    pw = orc.make_params(nx, ny, nz, 0.52, cs=0.1, fx=1e-6, bc=orc.WFB)
    pf = orc.make_params(nx, ny, nz, 0.52, cs=0.1, fx=1e-6, bc=orc.FREESLIP)
    ow, of = orc.Oracle(pw), orc.Oracle(pf)
    ow.set_state(f0)
    of.set_state(f0)
    rw, uxw, _, _ = ow.observe()
    rf, uxf, _, _ = of.observe()
    taux, _, _, _ = ow.wall()
    np.testing.assert_allclose(rw, rf, rtol=4e-16, atol=0)
    np.testing.assert_array_equal(uxw[:, 1:-1, :], uxf[:, 1:-1, :])
    np.testing.assert_allclose(uxw[:, 0, :] - uxf[:, 0, :], taux[0] / rw[:, 0, :], rtol=1e-9, atol=1e-18)
