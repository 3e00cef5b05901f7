"""Pins of the oracle's wall function (Eq. 16-17 and the Newton solve of Sec. 2.3)."""
import numpy as np
import pytest

KAPPA, B = 0.41, 5.5


def test_spalding_closed_form_matches_series(orc):
    # Eq. 16's bracket is the exponential series from its 4th term on.
    for up in [0.1, 1.0, 5.0, 12.0, 25.0]:
        k = KAPPA * up
        series = sum(k ** n / np.prod(np.arange(1, n + 1, dtype=float)) for n in range(4, 60))
        want = up + np.exp(-KAPPA * B) * series
        assert abs(orc.spalding_yplus(up) - want) <= 1e-12 * want


@pytest.mark.parametrize("yplus", np.geomspace(1e-3, 1e5, 41))
def test_inverse_profile_residual(orc, yplus):
    up = orc.spalding_uplus(yplus)
    assert abs(orc.spalding_yplus(up) - yplus) <= 1e-10 * yplus


def test_asymptotes(orc):
    # viscous sublayer: u+ -> y+
    for yp in [1e-3, 1e-2, 0.1]:
        assert abs(orc.spalding_uplus(yp) - yp) < 1e-4 * yp + 1e-12
    # log layer: u+ - (ln y+ / kappa + B) -> 0
    gaps = [abs(orc.spalding_uplus(yp) - (np.log(yp) / KAPPA + B)) for yp in [1e3, 1e4, 1e5]]
    assert gaps[0] > gaps[1] > gaps[2] and gaps[2] < 0.05


@pytest.mark.parametrize("U,y1,nu", [(1e-6, 1.0, 1e-4), (0.03, 1.0, 2.04e-5), (0.05, 1.0, 5.8e-6),
                                     (0.02, 0.5, 1e-4), (0.3, 1.0, 0.1), (0.2, 1.0, 1e-5)])
def test_newton_wall_solve(orc, U, y1, nu):
    """u_tau from the Newton solve satisfies Eq. 16 with y+ = y1 u_tau / nu and
    u+ = U / u_tau (Eq. 17) to 1e-10 relative."""
    ut, it = orc.wall_utau(U, y1, nu)
    assert ut > 0 and 1 <= it < 100
    yp, up = y1 * ut / nu, U / ut
    assert abs(orc.spalding_yplus(up) - yp) <= 1e-10 * yp


def test_newton_iterates_are_monotone(orc):
    """From u+_0 = sqrt(R) the iterates decrease monotonically to the root
    (H(p) = p Sp(p) - R is increasing and convex, and H(sqrt R) >= 0)."""
    for R in [1e-3, 1.0, 50.0, 1200.0, 4750.0, 2e4]:
        p = np.sqrt(R)
        ekb = np.exp(-KAPPA * B)
        for _ in range(200):
            k = KAPPA * p
            sp = p + ekb * (np.expm1(k) - k - k * k / 2 - k ** 3 / 6)
            dsp = 1 + KAPPA * ekb * (np.expm1(k) - k - k * k / 2)
            assert p * sp - R >= -1e-12 * R
            pn = p - (p * sp - R) / (sp + p * dsp)
            assert pn <= p * (1 + 1e-15)
            done = abs(pn - p) <= 1e-14 * pn
            p = pn
            if done:
                break
        ut, _ = orc.wall_utau(R * 1e-4, 1.0, 1e-4)   # same R = y1 U / nu
        assert abs(1e-4 * R / ut - p) <= 1e-12 * p


def test_iteration_cap_reports_failure(orc):
    # R = 1e5 needs more than 100 steps from sqrt(R): reported, not returned.
    ut, it = orc.wall_utau(1.0, 1.0, 1e-5, maxit=100)
    assert ut < 0 and it == 100


def test_zero_speed_gives_zero_stress(orc):
    ut, it = orc.wall_utau(0.0, 1.0, 1e-4)
    assert ut == 0.0 and it == 0


def test_wfb_stress_is_rho_utau_squared(orc):
    """tau_w = rho u_tau^2 (Eq. 17) with rho the local density."""
    p = orc.make_params(4, 4, 4, 0.51, fx=0.0)
    rng = np.random.default_rng(3)
    for _ in range(20):
        rho = rng.uniform(0.95, 1.05)
        u = np.array([rng.uniform(0.01, 0.08), 0.0, rng.uniform(-0.02, 0.02)])
        f = orc.feq(rho, u)
        _, rec, st, _ = orc.wfb_cell(p, 0, f)
        assert st == 0
        taux, tauz, ut, U = rec
        assert abs(np.hypot(taux, tauz) - rho * ut * ut) <= 1e-14 * rho * ut * ut
