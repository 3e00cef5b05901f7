"""ctypes wrapper of the FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the CPU-baseline leg of the benchmark may
import this module.  It shares nothing with the GPU library; states are
full populations f (not f - w) in the layout [a][z][y][x].
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

Q = 19
BB, WFB, FREESLIP = 0, 1, 2
BGK, MRT = 0, 1
# MRT rates of the non-hydrodynamic moments for D3Q19: energy, energy square,
# heat flux and third-order m moments as suggested by d'Humieres et al. (2002);
# the fourth-order normal stresses near the shear rate (1.99): a value fitted
# so that the channel runs reproduce the wall-law figures of Tables 2 and 3
# (the paper states none; the reference suggests 1.4)
MRT_RATES = dict(s_e=1.19, s_eps=1.4, s_q=1.2, s_pi=1.99, s_m=1.98)
OK, E_ARG, E_NONFINITE, E_NEWTON = 0, -1, -5, -6


class Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("bc", C.c_int32),
        ("tau0", C.c_double), ("cs", C.c_double), ("kappa", C.c_double),
        ("bconst", C.c_double), ("fx", C.c_double), ("y1", C.c_double),
        ("newton_tol", C.c_double), ("newton_maxit", C.c_int32),
        ("stats_every", C.c_int32), ("collision", C.c_int32),
        ("s_e", C.c_double), ("s_eps", C.c_double), ("s_q", C.c_double), ("s_pi", C.c_double),
        ("s_m", C.c_double), ("vd_aplus", C.c_double), ("vd_utau", C.c_double),
        ("wall_nodes", C.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("ORC_LIB_PATH")  # a planted-mistake build, loaded by the pin tests only
        if not path:
            if not os.path.exists(_build.LIB):
                _build.build()
            path = _build.LIB
        L = C.CDLL(path)
        dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
        ip = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
        i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
        PP = C.POINTER(Params)
        L.orc_tables.argtypes = [i32p, dp, i32p, i32p]
        L.orc_threads.restype = C.c_int32
        L.orc_threads.argtypes = []
        L.orc_set_threads.argtypes = [C.c_int32]
        L.orc_spalding_yplus.restype = C.c_double
        L.orc_spalding_yplus.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_spalding_uplus.restype = C.c_double
        L.orc_spalding_uplus.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_wall_utau.restype = C.c_double
        L.orc_wall_utau.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double,
                                    C.c_double, C.c_double, C.c_int, C.POINTER(C.c_int32)]
        L.orc_feq.argtypes = [C.c_double, dp, dp]
        L.orc_wall_tau.restype = C.c_int
        L.orc_wall_tau.argtypes = [PP, C.c_double, C.c_double, C.c_double, dp, C.POINTER(C.c_int32)]
        L.orc_wall_node_collide.argtypes = [PP, C.c_int, dp, C.c_double, C.c_double, dp]
        L.orc_get_wall_nodes.restype = C.c_int
        L.orc_get_wall_nodes.argtypes = [C.c_void_p, dp, dp]
        L.orc_set_wall_nodes.restype = C.c_int
        L.orc_set_wall_nodes.argtypes = [C.c_void_p, dp, dp]
        L.orc_wfb_cell.restype = C.c_int
        L.orc_wfb_cell.argtypes = [PP, C.c_int, dp, dp, C.POINTER(C.c_int32)]
        L.orc_collide_cell.argtypes = [PP, dp, dp, C.POINTER(C.c_double)]
        L.orc_collide_cell_at.argtypes = [PP, C.c_int, dp, dp, C.POINTER(C.c_double)]
        L.orc_mrt_basis.argtypes = [dp]
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [PP]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_set_param_bc.argtypes = [C.c_void_p, C.c_int32]
        L.orc_set_state.argtypes = [C.c_void_p, dp]
        L.orc_get_state.argtypes = [C.c_void_p, dp]
        L.orc_steps.restype = C.c_int64
        L.orc_steps.argtypes = [C.c_void_p]
        L.orc_max_newton_iters.restype = C.c_int32
        L.orc_max_newton_iters.argtypes = [C.c_void_p]
        L.orc_first_bad_step.restype = C.c_int64
        L.orc_first_bad_step.argtypes = [C.c_void_p]
        L.orc_initial_profile.argtypes = [PP, C.c_double, dp]
        L.orc_init_spalding.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_uint64]
        L.orc_step.restype = C.c_int
        L.orc_step.argtypes = [C.c_void_p, C.c_int64]
        L.orc_observe.restype = C.c_int
        L.orc_observe.argtypes = [C.c_void_p, dp, dp, dp, dp]
        L.orc_wall.restype = C.c_int
        L.orc_wall.argtypes = [C.c_void_p, dp, dp, dp, dp]
        L.orc_stats_sums.argtypes = [C.c_void_p, dp, C.POINTER(C.c_int64)]
        L.orc_stats_reset.argtypes = [C.c_void_p]
        L.orc_init_cells.restype = C.c_int
        L.orc_init_cells.argtypes = [PP, C.c_double, C.c_double, C.c_uint64, C.c_int64, ip, dp]
        L.orc_step_cells_table.restype = C.c_int
        L.orc_step_cells_table.argtypes = [PP, C.c_int64, ip, dp, C.c_int64, ip, dp, dp]
        L.orc_step1_cells.restype = C.c_int
        L.orc_step1_cells.argtypes = [PP, C.c_double, C.c_double, C.c_uint64, C.c_int64, ip, dp, dp]
        _lib = L
    return _lib


def threads():
    """Threads the oracle's loops use."""
    return lib().orc_threads()


def set_threads(n):
    lib().orc_set_threads(int(n))


def tables():
    """(e [19,3] int, w [19], opp [19], mirror_y [19]) as the oracle holds them."""
    e = np.zeros(57, np.int32)
    w = np.zeros(19)
    opp = np.zeros(19, np.int32)
    mir = np.zeros(19, np.int32)
    lib().orc_tables(e, w, opp, mir)
    return e.reshape(19, 3), w, opp, mir


def make_params(nx, ny, nz, tau0, cs=0.1, kappa=0.41, bconst=5.5, fx=0.0, bc=WFB,
                y1=1.0, newton_tol=1e-14, newton_maxit=100, stats_every=0, collision=BGK,
                rates=None, vd_aplus=0.0, vd_utau=0.0, wall_nodes=0):
    r = dict(MRT_RATES, **(rates or {}))
    return Params(nx, ny, nz, bc, tau0, cs, kappa, bconst, fx, y1, newton_tol,
                  newton_maxit, stats_every, collision, r["s_e"], r["s_eps"], r["s_q"], r["s_pi"],
                  r["s_m"], vd_aplus, vd_utau, int(wall_nodes))


# populations a wall node sends into the fluid, in the order of the wall-node arrays
IN_W = ((3, 7, 11, 14, 17), (4, 13, 18, 8, 12))


def wall_tau(params, rho, vx, vz):
    """Eq. 15-17 for a density and wall-parallel velocity: (tau_x, tau_z, u_tau, U), status."""
    rec = np.zeros(4)
    it = C.c_int32(0)
    st = lib().orc_wall_tau(C.byref(params), float(rho), float(vx), float(vz), rec, C.byref(it))
    return rec, st


def wall_node_collide(params, wall, f, taux, tauz):
    """The literal collision of a wall node (Eq. 14; Eq. 3 for bounce-back; Eq. 4
    for free-slip) on the 19 populations f that reached it."""
    out = np.zeros(19)
    lib().orc_wall_node_collide(C.byref(params), int(wall), np.ascontiguousarray(f, dtype=np.float64),
                                float(taux), float(tauz), out)
    return out


def spalding_yplus(uplus, kappa=0.41, b=5.5):
    return lib().orc_spalding_yplus(float(uplus), kappa, b)


def spalding_uplus(yplus, kappa=0.41, b=5.5):
    return lib().orc_spalding_uplus(float(yplus), kappa, b)


def wall_utau(U, y1, nu, kappa=0.41, b=5.5, tol=1e-14, maxit=100):
    it = C.c_int32(0)
    ut = lib().orc_wall_utau(float(U), float(y1), float(nu), kappa, b, tol, maxit, C.byref(it))
    return ut, it.value


def feq(rho, u):
    out = np.zeros(19)
    lib().orc_feq(float(rho), np.ascontiguousarray(u, dtype=np.float64), out)
    return out


def wfb_cell(params, wall, f):
    """Apply the WFB correction to a copy of f; returns (f_new, record, status, iters)."""
    f = np.array(f, dtype=np.float64)
    rec = np.zeros(4)
    it = C.c_int32(0)
    st = lib().orc_wfb_cell(C.byref(params), int(wall), f, rec, C.byref(it))
    return f, rec, st, it.value


def collide_cell(params, f, y=None):
    """Collision of one cell (row y for the van Driest damping; None: undamped)."""
    out = np.zeros(19)
    taue = C.c_double(0.0)
    f = np.ascontiguousarray(f, dtype=np.float64)
    if y is None:
        lib().orc_collide_cell(C.byref(params), f, out, C.byref(taue))
    else:
        lib().orc_collide_cell_at(C.byref(params), int(y), f, out, C.byref(taue))
    return out, taue.value


def mrt_basis():
    """The moment basis rows [19 moments, 19 velocities] as the oracle holds them."""
    m = np.zeros(19 * 19)
    lib().orc_mrt_basis(m)
    return m.reshape(19, 19)


def rule_m(ny, re_tau, ma, kappa=0.41, b=5.5, y1=1.0):
    """Workload parameters for a channel of ny layers (D = ny / 2) at Re_tau
    with centreline Mach number ma: returns dict(u_tau, nu0, tau0, fx, yplus1)."""
    D = ny / 2.0
    uc = ma / np.sqrt(3.0)
    u_tau = uc / spalding_uplus(re_tau, kappa, b)
    nu0 = u_tau * D / re_tau
    return dict(u_tau=u_tau, nu0=nu0, tau0=0.5 + 3.0 * nu0, fx=u_tau * u_tau / D,
                yplus1=y1 * u_tau / nu0)


class Oracle:
    """A channel held by the oracle (two FP64 population arrays)."""

    def __init__(self, params):
        self.params = params
        self.shape = (params.nz, params.ny, params.nx)
        self.ncell = params.nx * params.ny * params.nz
        self._h = lib().orc_create(C.byref(params))
        if not self._h:
            raise ValueError("oracle: invalid parameters")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    def set_bc(self, bc):
        self.params.bc = bc
        lib().orc_set_param_bc(self._h, bc)

    def set_state(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(19 * self.ncell)
        lib().orc_set_state(self._h, f)

    def state(self):
        out = np.zeros(19 * self.ncell)
        lib().orc_get_state(self._h, out)
        return out.reshape((19,) + self.shape)

    def init_spalding(self, u_tau, noise=0.05, seed=0):
        lib().orc_init_spalding(self._h, float(u_tau), float(noise), int(seed))

    def step(self, n=1):
        return lib().orc_step(self._h, int(n))

    @property
    def steps(self):
        return lib().orc_steps(self._h)

    @property
    def max_newton_iters(self):
        return lib().orc_max_newton_iters(self._h)

    @property
    def first_bad_step(self):
        return lib().orc_first_bad_step(self._h)

    def observe(self):
        """(rho, ux, uy, uz), each [nz, ny, nx]."""
        outs = [np.zeros(self.ncell) for _ in range(4)]
        st = lib().orc_observe(self._h, *outs)
        if st != OK:
            raise RuntimeError("oracle observe failed: %d" % st)
        return tuple(o.reshape(self.shape) for o in outs)

    def wall(self):
        """(tau_x, tau_z, u_tau, U), each [2, nz, nx]."""
        n = 2 * self.params.nx * self.params.nz
        outs = [np.zeros(n) for _ in range(4)]
        st = lib().orc_wall(self._h, *outs)
        if st != OK:
            raise RuntimeError("oracle wall failed: %d" % st)
        return tuple(o.reshape(2, self.params.nz, self.params.nx) for o in outs)

    def wall_mass_change(self):
        """Appendix B, Eq. B-1, per wall cell: the sum of the 19 populations after
        the WFB collision (Eq. 14) of the next step minus the sum before it, in
        FP64 over the full populations f, and the density before it.  The gather
        is the first-layer one of the halfway walls: in-domain populations from
        the neighbour, the wall-normal ones bounced back in place, the tangential
        diagonals mirrored (bounce-back walls: all bounced back).  Returns
        (dsum, rho), each [2, nz, nx], bottom wall first."""
        nx, ny, nz = self.params.nx, self.params.ny, self.params.nz
        bc = self.params.bc
        e, _, opp, mir = tables()
        f0 = self.state()
        dsum = np.zeros((2, nz, nx))
        rho = np.zeros((2, nz, nx))
        for wall, y in ((0, 0), (1, ny - 1)):
            for z in range(nz):
                for x in range(nx):
                    f = np.empty(Q)
                    for a in range(Q):
                        sy = y - e[a, 1]
                        if 0 <= sy < ny:
                            f[a] = f0[a, (z - e[a, 2]) % nz, sy, (x - e[a, 0]) % nx]
                        elif bc == BB or (e[a, 0] == 0 and e[a, 2] == 0):
                            f[a] = f0[opp[a], z, y, x]
                        else:
                            f[a] = f0[mir[a], (z - e[a, 2]) % nz, y, (x - e[a, 0]) % nx]
                    g = f
                    if bc == WFB:
                        g, _, st, _ = wfb_cell(self.params, wall, f)
                        if st != OK:
                            raise RuntimeError("oracle WFB failed: %d" % st)
                    s0 = 0.0
                    for a in range(Q):
                        s0 += f[a]
                    s1 = 0.0
                    for a in range(Q):
                        s1 += g[a]
                    dsum[wall, z, x] = s1 - s0
                    rho[wall, z, x] = s0
        return dsum, rho

    def wall_nodes(self):
        """(fw [2, 5, nz, nx]: what the wall nodes send into the fluid next step, in
        the direction order IN_W; urec [2, nz, nx, 3]: the first layer's rho, u_x,
        u_z of the latest step)."""
        nx, nz = self.params.nx, self.params.nz
        fw = np.zeros(2 * 5 * nz * nx)
        ur = np.zeros(2 * nz * nx * 3)
        st = lib().orc_get_wall_nodes(self._h, fw, ur)
        if st != OK:
            raise RuntimeError("oracle has no wall nodes")
        return fw.reshape(2, 5, nz, nx), ur.reshape(2, nz, nx, 3)

    def set_wall_nodes(self, fw, urec):
        """Sets the wall-node state (layouts of wall_nodes())."""
        st = lib().orc_set_wall_nodes(self._h, np.ascontiguousarray(fw, dtype=np.float64).reshape(-1),
                                      np.ascontiguousarray(urec, dtype=np.float64).reshape(-1))
        if st != OK:
            raise RuntimeError("oracle has no wall nodes")

    def stats_sums(self):
        out = np.zeros(8 * self.params.ny)
        ns = C.c_int64(0)
        lib().orc_stats_sums(self._h, out, C.byref(ns))
        return out.reshape(self.params.ny, 8), ns.value

    def stats_reset(self):
        lib().orc_stats_reset(self._h)


def initial_profile(params, u_tau):
    out = np.zeros(params.ny)
    lib().orc_initial_profile(C.byref(params), float(u_tau), out)
    return out


def init_cells(params, u_tau, noise, seed, cells):
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    out = np.zeros((len(cells), 19))
    st = lib().orc_init_cells(C.byref(params), float(u_tau), float(noise), int(seed), len(cells), cells, out.reshape(-1))
    if st != OK:
        raise RuntimeError("oracle init_cells failed: %d" % st)
    return out


def step1_cells(params, u_tau, noise, seed, cells):
    """Post-collision populations after one step, and observables (rho, u) of
    the initial state, at the given cell indices (x + nx (y + ny z))."""
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    out = np.zeros((len(cells), 19))
    mom = np.zeros((len(cells), 4))
    st = lib().orc_step1_cells(C.byref(params), float(u_tau), float(noise), int(seed), len(cells), cells,
                               out.reshape(-1), mom.reshape(-1))
    if st != OK:
        raise RuntimeError("oracle step1_cells failed: %d" % st)
    return out, mom


def neighbourhood(grid, cells):
    """The cells of the 3 x 3 x 3 neighbourhoods (x and z periodic, y clipped to
    the channel) of the given cells, ascending and unique."""
    nx, ny, nz = grid
    cells = np.asarray(cells, dtype=np.int64)
    x, y, z = cells % nx, (cells // nx) % ny, cells // (nx * ny)
    out = []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                yy = y + dy
                ok = (yy >= 0) & (yy < ny)
                out.append((((x + dx) % nx) + nx * (yy + ny * ((z + dz) % nz)))[ok])
    return np.unique(np.concatenate(out))


def step_cells_table(params, tab_cells, tab_f, cells):
    """One step at the given cells from a table of post-collision populations
    tab_f [k][19] of the cells tab_cells (ascending); returns the post-collision
    populations [n][19] and the observables (rho, u) [n][4] of the table's state."""
    tab_cells = np.ascontiguousarray(tab_cells, dtype=np.int64)
    tab_f = np.ascontiguousarray(tab_f, dtype=np.float64)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    out = np.zeros((len(cells), 19))
    mom = np.zeros((len(cells), 4))
    st = lib().orc_step_cells_table(C.byref(params), len(tab_cells), tab_cells, tab_f.reshape(-1), len(cells), cells,
                                    out.reshape(-1), mom.reshape(-1))
    if st != OK:
        raise RuntimeError("oracle step_cells_table failed: %d" % st)
    return out, mom
