"""Pins of the oracle's full step against closed forms and conservation laws.

- mass: streaming is a permutation and every collision conserves mass;
- x-momentum: each step adds exactly Fx per cell (Guo forcing) plus the
  wall force (WFB: the tau of Eq. 9; BB: momentum exchange; free-slip: 0);
- Poiseuille: the exact discrete solution of BGK + Guo + halfway bounce-back,
  a parabola plus a wall slip F(16 s^2 - 3)/(8 s), s = tau - 1/2, which
  vanishes at tau = 1/2 + sqrt(3)/4;
- free-slip: a uniform wall-parallel flow is a fixed point (Eq. 4);
- WFB force balance: in a laminar steady state the wall stress balances the
  body force, tau_x = -Fx D, and the wall record satisfies Spalding's law;
- Smagorinsky: the relaxation time solves the closure on a state of known
  non-equilibrium stress; Cs = 0 is plain BGK;
- force term: zeroth, first and second moments of Guo et al.'s term.
"""
import math

import numpy as np
import pytest


def _c1(orc, bc, tau=None, stats_every=0):
    rm = orc.rule_m(16, 640, 0.06)
    p = orc.make_params(32, 16, 16, rm["tau0"] if tau is None else tau, cs=0.1, fx=rm["fx"],
                        bc=bc, stats_every=stats_every)
    o = orc.Oracle(p)
    o.init_spalding(rm["u_tau"], 0.05, 0)
    return o, rm


def _xmom(orc, f):
    e, _, _, _ = orc.tables()
    return math.fsum((e[:, 0][:, None] * f.reshape(19, -1)).ravel())


@pytest.mark.parametrize("bc", [0, 1, 2])
def test_mass_conserved(orc, bc):
    o, _ = _c1(orc, bc)
    m0 = math.fsum(o.state().ravel())
    assert o.step(200) == 0
    m1 = math.fsum(o.state().ravel())
    assert abs(m1 - m0) <= 1e-12 * m0


@pytest.mark.parametrize("bc", [0, 1, 2])
def test_x_momentum_budget(orc, bc):
    o, rm = _c1(orc, bc)
    n = o.ncell
    for _ in range(15):
        p0 = _xmom(orc, o.state())
        taux, _, _, _ = o.wall()
        assert o.step(1) == 0
        p1 = _xmom(orc, o.state())
        want = n * rm["fx"] + math.fsum(taux.ravel())
        assert abs((p1 - p0) - want) <= 1e-9 * abs(want) + 1e-13 * abs(p0)
        if bc == 2:
            assert np.all(taux == 0.0)


def _poiseuille(orc, tau, ny, steps, F=1e-6):
    p = orc.make_params(1, ny, 1, tau, cs=0.0, fx=F, bc=orc.BB)
    o = orc.Oracle(p)
    nu, s = (tau - 0.5) / 3.0, tau - 0.5
    y = np.arange(ny) + 0.5
    exact = F / (2 * nu) * y * (ny - y) + F * (16 * s * s - 3) / (8 * s)
    f0 = np.stack([orc.feq(1.0, np.array([0.9 * u, 0.0, 0.0])) for u in exact], axis=1)
    o.set_state(f0.reshape(19, 1, ny, 1))
    assert o.step(steps) == 0
    _, ux, uy, uz = o.observe()
    return ux[0, :, 0], exact, F / (2 * nu) * y * (ny - y)


def test_poiseuille_exact_discrete_solution(orc):
    u, exact, parabola = _poiseuille(orc, 0.8, 32, 30000)
    assert np.abs(u - exact).max() <= 1e-10 * exact.max()
    assert np.abs(u - parabola).max() <= 1e-3 * parabola.max()


def test_poiseuille_slip_vanishes_at_magic_tau(orc):
    u, exact, parabola = _poiseuille(orc, 0.5 + math.sqrt(3.0) / 4.0, 16, 12000)
    assert np.abs(u - parabola).max() <= 1e-10 * parabola.max()


def test_freeslip_uniform_flow_is_a_fixed_point(orc):
    nx, ny, nz = 6, 5, 4
    f1 = orc.feq(1.0, np.array([0.04, 0.0, -0.03]))
    f0 = np.broadcast_to(f1[:, None, None, None], (19, nz, ny, nx)).copy()
    for bc, moves in ((orc.FREESLIP, False), (orc.BB, True)):
        o = orc.Oracle(orc.make_params(nx, ny, nz, 0.53, cs=0.1, fx=0.0, bc=bc))
        o.set_state(f0)
        assert o.step(25) == 0
        d = np.abs(o.state() - f0).max()
        if moves:
            assert d > 1e-4
        else:
            assert d <= 1e-15


def test_wfb_laminar_force_balance(orc):
    ny, F, tau = 16, 1e-6, 0.8
    o = orc.Oracle(orc.make_params(1, ny, 1, tau, cs=0.0, fx=F, bc=orc.WFB))
    f0 = np.stack([orc.feq(1.0, np.zeros(3))] * ny, axis=1)
    o.set_state(f0.reshape(19, 1, ny, 1))
    assert o.step(20000) == 0
    taux, tauz, ut, U = o.wall()
    rho, _, _, _ = o.observe()
    D = ny / 2.0
    nu = (tau - 0.5) / 3.0
    assert abs(taux.mean() + F * D) <= 1e-10 * F * D
    assert np.all(tauz == 0.0)
    for w, y in ((0, 0), (1, ny - 1)):
        utau, Uw = ut[w, 0, 0], U[w, 0, 0]
        assert abs(rho[0, y, 0] * utau ** 2 - F * D) <= 1e-10 * F * D
        yp = 1.0 * utau / nu
        assert abs(orc.spalding_yplus(Uw / utau) - yp) <= 1e-12 * yp


def test_smagorinsky_relaxation_time(orc):
    e, w, _, _ = orc.tables()
    rng = np.random.default_rng(21)
    for cs in (0.0, 0.1, 0.3):
        for _ in range(20):
            rho = rng.uniform(0.97, 1.03)
            u = rng.uniform(-0.05, 0.05, 3)
            P = rng.normal(0, 1e-4, (3, 3))
            P = P + P.T
            P -= np.trace(P) / 3.0 * np.eye(3)
            fneq = 4.5 * w * (np.einsum("ai,aj,ij->a", e, e, P) - np.trace(P) / 3.0)
            f = orc.feq(rho, u) + fneq
            tau0 = rng.uniform(0.5001, 0.9)
            p = orc.make_params(4, 4, 4, tau0, cs=cs, fx=0.0)
            out, taue = orc.collide_cell(p, f)
            Qn = math.sqrt(2.0 * np.sum(P * P))
            want = 0.5 * (tau0 + math.sqrt(tau0 ** 2 + 18.0 * cs * cs * Qn / rho))
            assert abs(taue - want) <= 1e-12 * want
            if cs == 0.0:
                assert taue == tau0
            fe = orc.feq(rho, u)
            np.testing.assert_allclose(out - fe, (1.0 - 1.0 / taue) * (f - fe), rtol=0, atol=5e-15)


def test_force_term_moments(orc):
    e, _, _, _ = orc.tables()
    rng = np.random.default_rng(23)
    for _ in range(30):
        f = orc.feq(rng.uniform(0.97, 1.03), rng.uniform(-0.05, 0.05, 3)) + rng.normal(0, 1e-4, 19)
        F = rng.uniform(-1e-4, 1e-4)
        tau = rng.uniform(0.51, 1.2)
        p = orc.make_params(4, 4, 4, tau, cs=0.0, fx=F)
        out, taue = orc.collide_cell(p, f)
        rho = f.sum()
        u = (e.T @ f + np.array([F / 2, 0, 0])) / rho
        force = out - f + (f - orc.feq(rho, u)) / tau
        beta = 1.0 - 1.0 / (2.0 * tau)
        Fv = np.array([F, 0.0, 0.0])
        assert abs(force.sum()) <= 1e-15
        np.testing.assert_allclose(e.T @ force, beta * Fv, rtol=0, atol=1e-15)
        np.testing.assert_allclose(np.einsum("ai,aj,a->ij", e, e, force),
                                   beta * (np.outer(u, Fv) + np.outer(Fv, u)), rtol=0, atol=1e-15)
        # and the whole step adds exactly F of momentum and no mass
        np.testing.assert_allclose(e.T @ (out - f), Fv, rtol=0, atol=2e-16)


def test_statistics_are_plane_sums_of_the_sampled_moments(orc):
    o, _ = _c1(orc, orc.WFB, tau=0.51, stats_every=2)
    want = np.zeros((16, 8))
    for t in range(1, 7):
        if t % 2 == 0:
            _, ux, uy, uz = o.observe()
            for k, q in enumerate((ux, uy, uz, ux * ux, uy * uy, uz * uz, ux * uy)):
                want[:, k] += q.sum(axis=(0, 2))
            want[:, 7] += 32 * 16
        assert o.step(1) == 0
    got, ns = o.stats_sums()
    assert ns == 3
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-16)
