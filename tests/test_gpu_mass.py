"""The Appendix B mass check on the device (Eq. B-1): the change of the
population sum that the wall correction makes, per wall cell, in the step's
own arithmetic.  The densities it reports against the oracle's; the changes
against the round-off bound of the four corrected populations and Table B-1's
largest order (FP64); exactly zero where the walls only permute."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_04352_amd as P
    return P


def _channel(P, store, bc, steps=31):
    from paper_2009_04352_amd import workloads as W
    p = W.params("c1")
    nx, ny, nz = p["grid"]
    ch = P.Channel(nx, ny, nz, p["tau0"], cs=p["cs"], fx=p["fx"], store=store, bc=bc)
    ch.init_spalding(p["u_tau"], p["noise"], p["seed"])
    ch.step(steps)
    return ch, p


@pytest.mark.parametrize("store", ("f64", "f32", "f16", "bf16"))
def test_wall_mass_change_is_roundoff(P, store):
    ch, p = _channel(P, store, "wfb")
    ds, rho = ch.wall_mass_change()
    assert ds.shape == (2, p["grid"][2], p["grid"][0]) and np.all(np.isfinite(ds))
    assert np.all(np.abs(rho - 1.0) < 0.05)
    # each of the four corrected populations and the two 19-term sums round once
    # per operation, in the step's precision, on values below |h| + |tau|/2 < 0.1
    eps = np.finfo(np.float64 if store == "f64" else np.float32).eps
    tx, tz, _, _ = ch.wall_shear()
    assert np.all(np.abs(ds) <= 42 * eps * (0.1 + np.abs(tx) + np.abs(tz)))
    if store == "f64":
        # Table B-1: at most of order 1e-14 of the mean population
        assert np.max(np.abs(ds) / (rho / 19.0)) <= 1e-14
    ch.close()


def test_wall_density_matches_the_oracle(P, orc):
    from gpu_common import oracle_for
    ch, p = _channel(P, "f64", "wfb")
    ds, rho = ch.wall_mass_change()
    o = oracle_for(orc, p["grid"], p["tau0"], p["cs"], p["fx"], "wfb")
    o.init_spalding(p["u_tau"], p["noise"], p["seed"])
    assert o.step(31) == 0
    dso, rhoo = o.wall_mass_change()
    assert np.max(np.abs(rho - rhoo)) <= 1e-13
    # both sides: zero or round-off of the same order (Table B-1)
    assert np.max(np.abs(dso) / (rhoo / 19.0)) <= 1e-14 and np.max(np.abs(ds) / (rho / 19.0)) <= 1e-14
    ch.close()


@pytest.mark.parametrize("bc", ("bb", "freeslip"))
def test_permuting_walls_change_nothing(P, bc):
    ch, _ = _channel(P, "f32", bc, steps=7)
    ds, rho = ch.wall_mass_change()
    assert np.all(ds == 0.0) and np.all(np.abs(rho - 1.0) < 0.05)
    ch.close()


def test_mass_check_statistics(P):
    from paper_2009_04352_amd import validation
    ch, _ = _channel(P, "f64", "wfb", steps=20)
    m = validation.mass_check(ch, 12)
    assert m["steps"] == 12 and 0.0 <= m["rate_nonzero"] <= 1.0 and 0.0 <= m["cell_rate_nonzero"] <= 1.0
    assert m["max_over_fbar"] <= m["cell_max_over_fbar"] <= 1e-14
    ch.close()
