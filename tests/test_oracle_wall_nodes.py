"""Pins of the oracle's wall-node picture (Sec. 2.1-2.2 read literally: the
wall grid is a lattice node at y = -1 and y = ny, one spacing from the first
fluid layer, where the reflections of Eq. 3, 4 and the WFB collision of
Eq. 14 happen; the stress comes from the first layer's velocity of the
previous step).

- the wall-node collision is Eq. 14 as printed (14a-b, the reversals and the
  copies of 14c; golden), bounce-back reverses everything (Eq. 3), free-slip
  is Eq. 14 without the stress (Eq. 4);
- brute force on a tiny grid: the populations the wall node sends are the
  first layer's populations of the previous step from x - e_b, reflected, and
  the first layer gathers them from x - e_a, two steps after they left (the
  one-step lag and the doubled tangential shift);
- mass of fluid plus wall nodes is conserved, and x-momentum changes each
  step by N Fx plus the stress of the wall-node collisions (Eq. 9, 12);
- steady states: bounce-back at wall nodes gives the exact discrete
  Poiseuille solution of halfway bounce-back (the lag does not matter in a
  steady state); uniform flow is a fixed point of free-slip wall nodes; the
  laminar WFB channel balances the body force with the wall stress.

wall_nodes = 2 takes the wall-node stress from the first layer's velocity of
the same step (the moments of the populations it gathers in that step)
instead of the previous one: the brute-force check recomputes that gather,
and the budgets and the steady state hold as for mode 1; for bounce-back and
free-slip, which apply no stress, the two modes agree bit for bit.
"""
import math

import numpy as np
import pytest

import golden_io


def _node_params(orc, nx, ny, nz, tau, bc, mode=1, **kw):
    return orc.make_params(nx, ny, nz, tau, bc=bc, wall_nodes=mode, **kw)


@pytest.mark.parametrize("wall", (0, 1))
def test_wall_node_collision_is_eq14_as_printed(orc, wall):
    e, _, opp, mir = orc.tables()
    rng = np.random.default_rng(3 + wall)
    f = rng.uniform(0.01, 0.1, 19)
    taux, tauz = 3e-5, -2e-5
    tau = {"x": taux, "z": tauz}
    p = _node_params(orc, 4, 4, 4, 0.52, orc.WFB)
    out = orc.wall_node_collide(p, wall, f, taux, tauz)
    m = (lambda a: a) if wall == 0 else (lambda a: int(mir[a]))
    shifted, reversed_ = golden_io.eq14()
    copies = golden_io.eq14_copies()
    seen = {m(0)}
    assert out[m(0)] == f[m(0)]                          # the rest population is not listed: unchanged
    for a, b, s, c in shifted:                           # 14a-b
        assert out[m(a)] == f[m(b)] + s * 0.5 * tau[c]
        seen.add(m(a))
    for a, b in reversed_:                               # 14c, reversals
        assert out[m(a)] == f[m(b)]
        seen.add(m(a))
    for a, b in copies:                                  # 14c, copies of the corrected values
        assert out[m(a)] == out[m(b)]
        seen.add(m(a))
    assert seen == set(range(19))
    # free-slip: the same without the stress; bounce-back: every population reversed
    pf = _node_params(orc, 4, 4, 4, 0.52, orc.FREESLIP)
    outf = orc.wall_node_collide(pf, wall, f, taux, tauz)
    for a, b, s, c in shifted:
        assert outf[m(a)] == f[m(b)]
    pb = _node_params(orc, 4, 4, 4, 0.52, orc.BB)
    outb = orc.wall_node_collide(pb, wall, f, taux, tauz)
    np.testing.assert_array_equal(outb, f[opp])
    # what the wall node sends into the fluid carries the mass it received (Eq. 12a)
    ins = list(orc.IN_W[wall])
    arr = [int(mir[a]) for a in ins]                     # the arrivals reflected into them
    assert abs(out[ins].sum() - f[arr].sum()) <= 4 * np.spacing(f[arr].sum())
    # and x-momentum changed by tau_x, z-momentum by tau_z (Eq. 9)
    dj = e[ins].T @ out[ins] - e[arr].T @ f[arr]
    np.testing.assert_allclose(dj, [taux, dj[1], tauz], rtol=0, atol=1e-17)


def _random_state(orc, shape, rng, u_scale=0.05):
    e, w, _, _ = orc.tables()
    nz, ny, nx = shape
    rho = 1.0 + rng.uniform(-0.02, 0.02, shape)
    u = rng.uniform(-u_scale, u_scale, (3,) + shape)
    u[0] += u_scale
    eu = np.einsum("ai,i...->a...", e.astype(np.float64), u)
    uu = (u * u).sum(axis=0)
    f = w[:, None, None, None] * rho[None] * (1 + 3 * eu + 4.5 * eu * eu - 1.5 * uu[None])
    return f * (1 + rng.uniform(-2e-3, 2e-3, f.shape))


@pytest.mark.parametrize("mode", (1, 2))
def test_lag_and_doubled_shift_on_a_tiny_grid(orc, mode):
    """Brute force: the wall nodes' outputs after one step are the reflected
    first-layer populations of the initial state from x - e_b, with the stress
    of the first layer at the node's column: its initial record (mode 1), or
    the moments of the populations it gathered in that step (mode 2); the
    first layer then gathers them from x - e_a."""
    e, _, opp, mir = orc.tables()
    nx, ny, nz = 5, 3, 4
    rng = np.random.default_rng(8)
    f0 = _random_state(orc, (nz, ny, nx), rng)
    p = _node_params(orc, nx, ny, nz, 0.52, orc.WFB, mode=mode, cs=0.1, fx=2e-6)
    o = orc.Oracle(p)
    o.set_state(f0)
    fw0, ur0 = o.wall_nodes()
    # the steady start: plain moments of the first layer, one wall-node collision of the initial state
    for w, y in ((0, 0), (1, ny - 1)):
        col = f0[:, :, y, :]
        r = col.sum(axis=0)
        np.testing.assert_allclose(ur0[w, :, :, 0], r, rtol=1e-15)
        np.testing.assert_allclose(ur0[w, :, :, 1], np.tensordot(e[:, 0], col, 1) / r, rtol=0, atol=1e-16)
        np.testing.assert_allclose(ur0[w, :, :, 2], np.tensordot(e[:, 2], col, 1) / r, rtol=0, atol=1e-16)
    assert o.step(1) == 0
    fw1, ur1 = o.wall_nodes()
    f1 = o.state()
    if mode == 2:
        # the record of step 1: moments (with the half force) of what the first
        # layer gathered, the fluid from f0 and the wall nodes' start outputs fw0
        for w, y in ((0, 0), (1, ny - 1)):
            for z in range(nz):
                for x in range(nx):
                    f = np.empty(19)
                    for a in range(19):
                        sy = y - e[a, 1]
                        sx, sz = (x - e[a, 0]) % nx, (z - e[a, 2]) % nz
                        f[a] = f0[a, sz, sy, sx] if 0 <= sy < ny else fw0[w, list(orc.IN_W[w]).index(a), sz, sx]
                    r = f.sum()
                    assert abs(ur1[w, z, x, 0] - r) <= 1e-15
                    assert abs(ur1[w, z, x, 1] - (e[:, 0] @ f + 0.5 * p.fx) / r) <= 1e-16
                    assert abs(ur1[w, z, x, 2] - (e[:, 2] @ f) / r) <= 1e-16
    urs = ur0 if mode == 1 else ur1
    shifted, _ = golden_io.eq14()
    sgn = {a: (s, c) for a, _, s, c in shifted}
    for w, y in ((0, 0), (1, ny - 1)):
        for z in range(nz):
            for x in range(nx):
                rec, st = orc.wall_tau(p, *urs[w, z, x])
                assert st == 0
                for k, a in enumerate(orc.IN_W[w]):
                    b = int(mir[a])                                  # the arrival reflected into a
                    src = f0[b, (z - e[b, 2]) % nz, y, (x - e[b, 0]) % nx]
                    a0 = a if w == 0 else int(mir[a])               # the bottom-wall name of a
                    add = 0.0
                    if a0 in sgn:
                        s, c = sgn[a0]
                        add = s * 0.5 * (rec[0] if c == "x" else rec[1])
                    assert fw1[w, k, z, x] == src + add, (w, k, z, x)
    # the next gather: from the wall node at x - e_a, i.e. two cells upstream of where it left
    rho, ux, uy, uz = o.observe()
    for w, y in ((0, 0), (1, ny - 1)):
        for z in range(nz):
            for x in range(nx):
                f = np.empty(19)
                for a in range(19):
                    sy = y - e[a, 1]
                    sx, sz = (x - e[a, 0]) % nx, (z - e[a, 2]) % nz
                    if 0 <= sy < ny:
                        f[a] = f1[a, sz, sy, sx]
                    else:
                        f[a] = fw1[w, list(orc.IN_W[w]).index(a), sz, sx]
                r = f.sum()
                assert abs(rho[z, y, x] - r) <= 1e-15
                want = (e.T @ f + np.array([0.5 * p.fx, 0.0, 0.0])) / r
                np.testing.assert_allclose([ux[z, y, x], uy[z, y, x], uz[z, y, x]], want, rtol=0, atol=1e-16)


def _totals(orc, o):
    e, _, _, _ = orc.tables()
    f = o.state().reshape(19, -1)
    fw, _ = o.wall_nodes()
    m = math.fsum(f.ravel()) + math.fsum(fw.ravel())
    px = math.fsum((e[:, 0][:, None] * f).ravel())
    for w in (0, 1):
        for k, a in enumerate(orc.IN_W[w]):
            px += math.fsum((e[a, 0] * fw[w, k]).ravel())
    return m, px


@pytest.mark.parametrize("mode", (1, 2))
@pytest.mark.parametrize("bc", (0, 1, 2))
def test_mass_and_x_momentum_of_fluid_and_wall_nodes(orc, bc, mode):
    """x-momentum of fluid plus wall nodes changes by N Fx plus the stress of
    the step's wall-node collisions: for WFB from the record before the step
    (mode 1) or from the one the step computed (mode 2); for bounce-back the
    momentum exchange of the populations waiting at the nodes."""
    nx, ny, nz = 6, 5, 4
    rng = np.random.default_rng(30 + bc)
    p = _node_params(orc, nx, ny, nz, 0.5003, bc, mode=mode, cs=0.1, fx=3e-6)
    o = orc.Oracle(p)
    o.set_state(_random_state(orc, (nz, ny, nx), rng))
    m0, _ = _totals(orc, o)
    for _ in range(6):
        _, p0 = _totals(orc, o)
        taux, _, _, _ = o.wall()
        assert o.step(1) == 0
        if mode == 2 and bc == orc.WFB:
            taux, _, _, _ = o.wall()   # the WFB stress of the step's own record
        m1, p1 = _totals(orc, o)
        want = nx * ny * nz * p.fx + math.fsum(taux.ravel())
        assert abs((p1 - p0) - want) <= 1e-9 * abs(want) + 1e-13 * abs(p0)
        if bc == orc.FREESLIP:
            assert np.all(taux == 0.0)
    assert o.step(30) == 0
    m1, _ = _totals(orc, o)
    assert abs(m1 - m0) <= 1e-13 * m0


def test_bounce_back_nodes_reach_the_exact_poiseuille_solution(orc):
    """Steady flow does not see the lag: bounce-back at wall nodes converges to
    the exact discrete solution of halfway bounce-back (slip
    F (16 s^2 - 3) / (8 s), s = tau - 1/2, walls at y = -1/2 and ny - 1/2)."""
    tau, ny, F = 0.8, 8, 1e-6
    p = _node_params(orc, 1, ny, 1, tau, orc.BB, cs=0.0, fx=F)
    o = orc.Oracle(p)
    nu, s = (tau - 0.5) / 3.0, tau - 0.5
    y = np.arange(ny) + 0.5
    exact = F / (2 * nu) * y * (ny - y) + F * (16 * s * s - 3) / (8 * s)
    f0 = np.stack([orc.feq(1.0, np.array([0.9 * u, 0.0, 0.0])) for u in exact], axis=1)
    o.set_state(f0.reshape(19, 1, ny, 1))
    assert o.step(6000) == 0
    _, ux, _, _ = o.observe()
    assert np.abs(ux[0, :, 0] - exact).max() <= 1e-10 * exact.max()


def test_uniform_flow_is_a_fixed_point_of_free_slip_nodes(orc):
    nx, ny, nz = 6, 5, 4
    f1 = orc.feq(1.0, np.array([0.04, 0.0, -0.03]))
    f0 = np.broadcast_to(f1[:, None, None, None], (19, nz, ny, nx)).copy()
    for bc, moves in ((orc.FREESLIP, False), (orc.BB, True)):
        o = orc.Oracle(_node_params(orc, nx, ny, nz, 0.53, bc, cs=0.1, fx=0.0))
        o.set_state(f0)
        assert o.step(25) == 0
        d = np.abs(o.state() - f0).max()
        if moves:
            assert d > 1e-4
        else:
            assert d <= 1e-15


@pytest.mark.parametrize("mode", (1, 2))
def test_wfb_nodes_laminar_force_balance(orc, mode):
    """The steady laminar channel with WFB wall nodes: the wall stress of both
    walls balances the body force on the ny fluid layers, mean tau_x = -F ny / 2,
    and the stress is Spalding's law at the first layer (y+ = y1 u_tau / nu)."""
    ny, F, tau = 8, 1e-6, 0.8
    o = orc.Oracle(_node_params(orc, 1, ny, 1, tau, orc.WFB, mode=mode, cs=0.0, fx=F))
    f0 = np.stack([orc.feq(1.0, np.zeros(3))] * ny, axis=1)
    o.set_state(f0.reshape(19, 1, ny, 1))
    assert o.step(8000) == 0
    taux, tauz, ut, U = o.wall()
    _, urec = o.wall_nodes()
    half = F * ny / 2.0
    nu = (tau - 0.5) / 3.0
    assert abs(taux.mean() + half) <= 1e-10 * half
    assert np.all(tauz == 0.0)
    for w in (0, 1):
        utau, Uw = ut[w, 0, 0], U[w, 0, 0]
        assert abs(urec[w, 0, 0, 0] * utau ** 2 - half) <= 1e-10 * half
        assert abs(Uw - abs(urec[w, 0, 0, 1])) <= 1e-16
        yp = 1.0 * utau / nu
        assert abs(orc.spalding_yplus(Uw / utau) - yp) <= 1e-12 * yp


def test_cell_paths_reject_wall_nodes(orc):
    p = _node_params(orc, 4, 4, 4, 0.52, orc.WFB)
    with pytest.raises(RuntimeError):
        orc.step1_cells(p, 0.01, 0.05, 0, np.arange(4, dtype=np.int64))


@pytest.mark.parametrize("bc", (0, 2))
def test_modes_agree_without_stress(orc, bc):
    """Bounce-back and free-slip wall nodes apply no stress: the two stress
    timings give the same states and wall nodes bit for bit."""
    nx, ny, nz = 6, 5, 4
    f0 = _random_state(orc, (nz, ny, nx), np.random.default_rng(40 + bc))
    out = []
    for mode in (1, 2):
        o = orc.Oracle(_node_params(orc, nx, ny, nz, 0.51, bc, mode=mode, cs=0.1, fx=2e-6))
        o.set_state(f0)
        assert o.step(9) == 0
        out.append((o.state(), o.wall_nodes()[0]))
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])
