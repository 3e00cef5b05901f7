"""Pins of the oracle's D3Q19 tables and equilibrium (Table A-1, Eq. 2, Eq. 10-11).

The oracle's tables must reproduce the transcribed Table A-1 and every
printed moment sum of Eq. 10-11; the equilibrium must have the textbook
moments of Qian et al. (1992), which Eq. 2 relies on.
"""
import numpy as np

import golden_io


def test_velocities_match_table_a1(orc):
    e, w, opp, mir = orc.tables()
    np.testing.assert_array_equal(e, golden_io.table_a1())


def test_printed_moment_sums_match_velocities(orc):
    e, _, _, _ = orc.tables()
    comp = {"x": 0, "y": 1, "z": 2}
    for eq, mom, coef, _ in golden_io.moment_sums():
        want = np.ones(19, dtype=np.int64) if mom == "rho" else e[:, comp[mom]]
        np.testing.assert_array_equal(coef, want, err_msg=eq)


def test_eq11_revises_exactly_the_bottom_in_pointing_diagonals(orc):
    e, _, _, _ = orc.tables()
    diag_in = {a for a in range(19) if e[a, 1] == 1 and (e[a, 0] != 0 or e[a, 2] != 0)}
    for eq, _, _, revised in golden_io.moment_sums():
        if eq.startswith("11"):
            assert revised <= diag_in
    assert diag_in == {7, 11, 14, 17}


def test_opposite_and_mirror_are_involutions(orc):
    e, _, opp, mir = orc.tables()
    for a in range(19):
        assert opp[opp[a]] == a and mir[mir[a]] == a
        np.testing.assert_array_equal(e[opp[a]], -e[a])
        np.testing.assert_array_equal(e[mir[a]], e[a] * np.array([1, -1, 1]))
        assert opp[mir[a]] == mir[opp[a]]


def test_mirror_pairs_are_those_of_eq14(orc):
    _, _, opp, mir = orc.tables()
    shifted, reversed_ = golden_io.eq14()
    for a, b, _, _ in shifted:
        assert mir[b] == a          # the reflected partner of Eq. 14a-b
    for a, b in reversed_:
        assert opp[a] == b          # the axis reversals of Eq. 14c


def test_wall_in_pointing_sets(orc):
    e, _, _, _ = orc.tables()
    assert {a for a in range(19) if e[a, 1] == 1} == {3, 7, 11, 14, 17}
    assert {a for a in range(19) if e[a, 1] == -1} == {4, 8, 12, 13, 18}


def test_weights_and_isotropy(orc):
    e, w, _, _ = orc.tables()
    assert abs(w.sum() - 1.0) < 1e-15
    np.testing.assert_allclose(np.einsum("a,ai->i", w, e), 0.0, atol=1e-16)
    np.testing.assert_allclose(np.einsum("a,ai,aj->ij", w, e, e), np.eye(3) / 3.0, atol=1e-16)
    # fourth moment: sum w e_i e_j e_k e_l = (d_ij d_kl + d_ik d_jl + d_il d_jk) / 9
    m4 = np.einsum("a,ai,aj,ak,al->ijkl", w, e, e, e, e)
    d = np.eye(3)
    want = (np.einsum("ij,kl->ijkl", d, d) + np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d)) / 9.0
    np.testing.assert_allclose(m4, want, atol=1e-16)


def test_equilibrium_moments(orc):
    """Eq. 2 on the equilibrium: sum f = rho, sum e f = rho u,
    sum e e f = rho/3 I + rho u u (so p = rho e_s^2 with e_s^2 = 1/3)."""
    e, _, _, _ = orc.tables()
    rng = np.random.default_rng(7)
    for _ in range(50):
        rho = rng.uniform(0.8, 1.2)
        u = rng.uniform(-0.1, 0.1, 3)
        f = orc.feq(rho, u)
        assert abs(f.sum() - rho) <= 1e-15 * rho * 4
        np.testing.assert_allclose(e.T @ f, rho * u, atol=4e-16)
        pi = np.einsum("ai,aj,a->ij", e, e, f)
        np.testing.assert_allclose(pi, rho / 3.0 * np.eye(3) + rho * np.outer(u, u), atol=4e-16)
