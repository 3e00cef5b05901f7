"""Pins of the oracle's MRT collision in whole flows.

- Poiseuille flow with halfway bounce-back in the two-relaxation-time limit
  (odd rates s-, even rates s+ = 1/tau): the wall slip is
  F (16 L - 3) / (8 L+), L = L+ L-, L+- = 1/s+- - 1/2, exact zero slip at
  L = 3/16;
- a turbulent channel start with MRT and van Driest damping conserves mass
  and its x-momentum changes by N Fx plus the wall force each step (WFB:
  the stress of Eq. 9; bounce-back: the momentum exchange).
"""
import math

import numpy as np
import pytest


def _poiseuille(orc, tau, s_odd, ny, steps, F=1e-6):
    # the two-relaxation-time limit: every odd rate s_odd, every even one 1/tau
    w = 1.0 / tau
    p = orc.make_params(1, ny, 1, tau, cs=0.0, fx=F, bc=orc.BB, collision=orc.MRT,
                        rates=dict(s_q=s_odd, s_m=s_odd, s_e=w, s_eps=w, s_pi=w))
    o = orc.Oracle(p)
    nu = (tau - 0.5) / 3.0
    y = np.arange(ny) + 0.5
    parabola = F / (2 * nu) * y * (ny - y)
    f0 = np.stack([orc.feq(1.0, np.array([0.9 * u, 0.0, 0.0])) for u in parabola], axis=1)
    o.set_state(f0.reshape(19, 1, ny, 1))
    assert o.step(steps) == 0
    _, ux, _, _ = o.observe()
    return ux[0, :, 0], parabola


@pytest.mark.parametrize("tau,s_odd", [(0.8, 1.2), (0.7, 1.5)])
def test_poiseuille_slip(orc, tau, s_odd):
    F = 1e-6
    u, parabola = _poiseuille(orc, tau, s_odd, 8, 6000, F)
    lp, lm = tau - 0.5, 1.0 / s_odd - 0.5
    slip = F * (16 * lp * lm - 3) / (8 * lp)
    assert np.abs(u - (parabola + slip)).max() <= 1e-10 * parabola.max()


def test_poiseuille_exact_at_magic_product(orc):
    tau = 0.6                                  # L+ = 0.1: L- = 1.875 gives L = 3/16
    u, parabola = _poiseuille(orc, tau, 1.0 / (1.875 + 0.5), 8, 9000)
    assert np.abs(u - parabola).max() <= 1e-10 * parabola.max()


def test_mrt_channel_conserves_mass_and_momentum_budget(orc):
    rm = orc.rule_m(16, 640, 0.06)
    for bc in (orc.BB, orc.WFB):
        o = orc.Oracle(orc.make_params(16, 16, 8, rm["tau0"], cs=0.1, fx=rm["fx"], bc=bc, collision=orc.MRT,
                                       vd_aplus=26.0))
        o.init_spalding(rm["u_tau"], 0.05, 0)
        e, _, _, _ = orc.tables()
        m0 = math.fsum(o.state().ravel())
        for _ in range(5):
            p0 = math.fsum((e[:, 0][:, None] * o.state().reshape(19, -1)).ravel())
            taux, _, _, _ = o.wall()
            assert o.step(1) == 0
            p1 = math.fsum((e[:, 0][:, None] * o.state().reshape(19, -1)).ravel())
            want = o.ncell * rm["fx"] + math.fsum(taux.ravel())   # BB: the momentum-exchange force
            assert abs((p1 - p0) - want) <= 1e-9 * abs(want) + 1e-13 * abs(p0)
        assert abs(math.fsum(o.state().ravel()) - m0) <= 1e-12 * m0
