"""Pins of the oracle's MRT collision (the paper's collision operator,
Sec. 3.1, after d'Humieres et al. 2002) and of the van Driest damping.

- the moment basis is orthogonal over the 19 velocities, its rows 0, 3, 5, 7
  are the conserved density and momentum, and the squared row norms are the
  ones of that basis;
- every non-conserved row is an eigenvector of the collision: a state off
  equilibrium in moment k alone relaxes by (1 - s_k) in that moment only,
  with s_k the rate of its class (stress at 1/tau, the others at theirs);
- with all rates equal MRT is BGK (to rounding), with the force term too;
- mass is conserved and the force adds exactly F of momentum per cell;
- van Driest: no damping for A+ -> 0 and no eddy viscosity for A+ -> inf,
  damping symmetric in the two walls and growing towards them.
(Flows with MRT: test_oracle_mrt_flows.py.)
"""
import numpy as np
import pytest

NORMS = [19, 2394, 252, 10, 40, 10, 40, 10, 40, 36, 72, 12, 24, 4, 4, 4, 8, 8, 8]
# the rate class of each moment: 'w' = 1/tau (stress and conserved), else the key
CLASS = ["w", "s_e", "s_eps", "w", "s_q", "w", "s_q", "w", "s_q", "w", "s_pi", "w", "s_pi", "w", "w", "w",
         "s_m", "s_m", "s_m"]


def test_moment_basis_is_orthogonal(orc):
    M = orc.mrt_basis()
    e, _, _, _ = orc.tables()
    G = M @ M.T
    assert np.array_equal(G, np.diag(NORMS).astype(float))
    assert np.all(M[0] == 1.0)
    for k, d in ((3, 0), (5, 1), (7, 2)):
        assert np.array_equal(M[k], e[:, d].astype(float))


@pytest.mark.parametrize("k", [1, 2, 4, 6, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18])
def test_each_moment_relaxes_at_its_rate(orc, k):
    M = orc.mrt_basis()
    tau = 0.7
    rates = dict(s_e=1.19, s_eps=1.4, s_q=1.2, s_pi=1.35, s_m=1.98)
    p = orc.make_params(2, 2, 2, tau, cs=0.0, fx=0.0, collision=orc.MRT, rates=rates)
    fe = orc.feq(1.03, np.array([0.04, -0.02, 0.01]))
    d = 1e-3 * M[k] / NORMS[k]          # moment k of d is 1e-3, all others 0
    out, _ = orc.collide_cell(p, fe + d)
    s = 1.0 / tau if CLASS[k] == "w" else rates[CLASS[k]]
    want = fe + (1.0 - s) * d
    assert np.abs(out - want).max() <= 1e-15


def test_equal_rates_give_bgk(orc):
    rng = np.random.default_rng(3)
    for tau in (0.52, 0.6, 1.3):
        w = 1.0 / tau
        pb = orc.make_params(2, 2, 2, tau, cs=0.0, fx=2e-5)
        pm = orc.make_params(2, 2, 2, tau, cs=0.0, fx=2e-5, collision=orc.MRT,
                             rates=dict(s_e=w, s_eps=w, s_q=w, s_pi=w, s_m=w))
        for _ in range(5):
            f = orc.feq(1.0 + rng.uniform(-0.02, 0.02), rng.uniform(-0.05, 0.05, 3)) * (1 + rng.uniform(-0.01, 0.01, 19))
            ob, _ = orc.collide_cell(pb, f)
            om, _ = orc.collide_cell(pm, f)
            assert np.abs(ob - om).max() <= 4e-16


def test_mass_and_force(orc):
    e, _, _, _ = orc.tables()
    rng = np.random.default_rng(4)
    p = orc.make_params(2, 2, 2, 0.51, cs=0.1, fx=3e-5, collision=orc.MRT)
    for _ in range(5):
        f = orc.feq(1.0 + rng.uniform(-0.02, 0.02), rng.uniform(-0.05, 0.05, 3)) * (1 + rng.uniform(-0.01, 0.01, 19))
        out, _ = orc.collide_cell(p, f)
        # to rounding: sums of 19 terms below 0.4 through the two transforms
        assert abs(out.sum() - f.sum()) <= 2e-15
        dj = e.T.astype(float) @ (out - f)
        assert abs(dj[0] - 3e-5) <= 2e-15 and abs(dj[1]) <= 2e-15 and abs(dj[2]) <= 2e-15


def _sheared(orc):
    return orc.feq(1.0, np.array([0.03, 0.0, 0.0])) + 2e-2 * orc.mrt_basis()[13] / 4.0   # p_xy off equilibrium


@pytest.mark.parametrize("coll", ["BGK", "MRT"])
def test_van_driest_limits(orc, coll):
    c = getattr(orc, coll)
    ny, tau, fx = 32, 0.5005, 1e-6
    f = _sheared(orc)
    plain = orc.make_params(4, ny, 4, tau, cs=0.1, fx=fx, collision=c)
    _, t_plain = orc.collide_cell(plain, f)
    assert t_plain > tau + 1e-3                 # the SGS viscosity is there
    tiny = orc.make_params(4, ny, 4, tau, cs=0.1, fx=fx, collision=c, vd_aplus=1e-300)
    huge = orc.make_params(4, ny, 4, tau, cs=0.1, fx=fx, collision=c, vd_aplus=1e300)
    for y in (0, 3, ny // 2):
        assert orc.collide_cell(tiny, f, y)[1] == t_plain
        assert abs(orc.collide_cell(huge, f, y)[1] - tau) <= 1e-15
    vd = orc.make_params(4, ny, 4, tau, cs=0.1, fx=fx, collision=c, vd_aplus=26.0)
    t = [orc.collide_cell(vd, f, y)[1] for y in range(ny)]
    assert all(t[y] == t[ny - 1 - y] for y in range(ny))
    assert all(t[y] < t[y + 1] for y in range(ny // 2 - 1))
    assert tau < t[0] and t[ny // 2] < t_plain
