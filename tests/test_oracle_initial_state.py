"""Pins of the oracle's initial state (the input recipe of every workload):
the splitmix64 draws match the generator's published reference outputs, the
noise of cell c and component i comes from draw 3 c + i, and the streamwise
profile satisfies Spalding's law (Eq. 16) at the distance d = min(y, ny-1-y) + y1."""
import numpy as np

M64 = (1 << 64) - 1


def splitmix64(seed, k):
    """Output k (0-based) of splitmix64 from state `seed` (Steele, Lea & Flood 2014)."""
    z = (seed + (k + 1) * 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def test_splitmix64_reference_outputs():
    # the first outputs of the generator started from state 0
    assert [splitmix64(0, k) for k in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def _initial_velocities(orc, grid, u_tau, noise, seed, tau=0.51, y1=1.0):
    nx, ny, nz = grid
    p = orc.make_params(nx, ny, nz, tau, y1=y1)
    cells = np.arange(nx * ny * nz, dtype=np.int64)
    f = orc.init_cells(p, u_tau, noise, seed, cells)          # [cell][a]
    e = orc.tables()[0].astype(np.float64)
    rho = f.sum(axis=1)
    u = (f @ e) / rho[:, None]
    return p, cells, rho, u


def test_initial_state_is_equilibrium_at_unit_density(orc):
    _, _, rho, _ = _initial_velocities(orc, (8, 6, 4), 0.01, 0.05, 3)
    assert np.allclose(rho, 1.0, rtol=0, atol=1e-15)


def test_noise_of_each_component_is_its_own_draw(orc):
    grid = (8, 6, 4)
    nx, ny, nz = grid
    u_tau, noise, seed = 0.01, 0.05, 7
    p, cells, _, u = _initial_velocities(orc, grid, u_tau, noise, seed)
    prof = orc.initial_profile(p, u_tau)
    y = (cells // nx) % ny
    up = prof[y]
    d = np.stack([u[:, 0] / up - 1.0, u[:, 1] / up, u[:, 2] / up], axis=1)
    want = np.array([[noise * (2.0 * ((splitmix64(seed, 3 * int(c) + i) >> 11) / 2.0 ** 53) - 1.0) for i in range(3)]
                     for c in cells])
    assert np.all(np.abs(d - want) <= 1e-12)


def test_initial_profile_satisfies_spalding_at_the_layer_distance(orc):
    ny, y1, tau, u_tau = 16, 1.0, 0.51, 0.02
    p = orc.make_params(4, ny, 4, tau, y1=y1)
    prof = orc.initial_profile(p, u_tau)
    nu0 = (tau - 0.5) / 3.0
    for y in range(ny):
        dist = min(y, ny - 1 - y) + y1
        yplus = dist * u_tau / nu0
        assert abs(orc.spalding_yplus(prof[y] / u_tau) - yplus) <= 1e-11 * yplus, y
