"""The profile metrics of Eq. 19 and Eq. 20 on profiles of known answer."""
import math

import numpy as np
import pytest

from paper_2009_04352_amd.channel import spalding_uplus
from paper_2009_04352_amd.validation import profile_metrics


def _profile(ny, u_tau, nu0, uplus_of):
    d = np.minimum(np.arange(ny), ny - 1 - np.arange(ny)) + 1.0
    return np.array([u_tau * uplus_of(v * u_tau / nu0) for v in d])


def test_spalding_profile_has_zero_error():
    u_tau, nu0 = 2e-3, 1e-4           # y+ from 20 to 1280 over 64 layers
    m = profile_metrics(_profile(128, u_tau, nu0, spalding_uplus), u_tau, nu0)
    assert m["eps_buffer"] <= 1e-14 and m["eps_log"] <= 1e-14 and m["eps_all"] <= 1e-14
    assert len(m["yplus"]) == 64 and abs(m["yplus"][0] - 20.0) <= 1e-12


def test_scaled_profile_error_is_the_scale():
    u_tau, nu0 = 2e-3, 1e-4
    m = profile_metrics(1.03 * _profile(128, u_tau, nu0, spalding_uplus), u_tau, nu0)
    for k in ("eps_buffer", "eps_log", "eps_all"):
        assert abs(m[k] - 0.03) <= 1e-12


def test_log_law_intercept():
    u_tau, nu0, b0 = 2e-3, 1e-4, 6.5
    m = profile_metrics(_profile(128, u_tau, nu0, lambda yp: math.log(yp) / 0.41 + b0), u_tau, nu0)
    assert abs(m["b"] - b0) <= 1e-12


def test_halves_are_folded():
    u_tau, nu0 = 2e-3, 1e-4
    u = _profile(128, u_tau, nu0, spalding_uplus)
    skew = np.linspace(-1.0, 1.0, 128) * 1e-3 * u.max()     # antisymmetric: cancels in the fold
    m = profile_metrics(u + skew, u_tau, nu0)
    assert m["eps_all"] <= 1e-12


def test_mass_check_aggregates_eq_b1():
    """Eq. B-1 averages the per-cell change over every wall cell of both walls;
    Table B-1 counts the steps whose average is not zero and takes the largest
    |average| over the mean population rho / 19.  A stand-in channel hands out
    known per-cell changes."""
    from paper_2009_04352_amd import validation

    class Fake:
        def __init__(self):
            self.k = 0
            self.steps = 0

        def wall_mass_change(self):
            ds = np.zeros((2, 2, 3))
            if self.k == 1:
                ds[0, 0, 0], ds[1, 1, 2] = 3e-17, -1e-17   # average 2e-17 / 12
            elif self.k == 2:
                ds[0, 1, 1], ds[1, 0, 0] = 4e-17, -4e-17   # cancels: average zero
            return ds, np.full((2, 2, 3), 0.95)

        def step(self, n):
            self.k += 1
            self.steps += n

    ch = Fake()
    m = validation.mass_check(ch, 4)
    assert ch.steps == 4 and m["steps"] == 4
    assert m["rate_nonzero"] == 0.25                       # only the second step
    assert m["max_over_fbar"] == pytest.approx((2e-17 / 12) / (0.95 / 19), rel=1e-12)
    assert m["cell_rate_nonzero"] == 4 / 48
    assert m["cell_max_over_fbar"] == pytest.approx(4e-17 / (0.95 / 19), rel=1e-12)


def test_table1_cases_match_the_paper():
    """The validation cases are Table 1's: grid, Re_tau, Ma_LB, D = ny / 2 equal
    to the resolution column, and the first-layer y+ of the Rule-M parameters
    equal to the printed one (to the table's rounding)."""
    import golden_io
    from paper_2009_04352_amd import workloads as W
    rows = golden_io.table1()
    assert sorted(r["case"] for r in rows) == sorted(W.TABLE1)
    for r in rows:
        c = W.TABLE1[r["case"]]
        assert c["grid"] == (r["nx"], r["ny"], r["nz"]) and c["re_tau"] == r["re_tau"] and c["ma"] == r["ma"]
        assert r["ny"] // 2 == r["res"]
        p = W.params(r["case"])
        assert abs(p["yplus1"] - r["yplus"]) <= 0.5
