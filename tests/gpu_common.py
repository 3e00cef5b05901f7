"""Shared helpers of the GPU tests: oracle set-up, store rounding, tolerances.

Tolerances are derived from the arithmetic (see test docstrings): the GPU
result of one step, stored in format T, may differ from the FP64 oracle by
the final rounding to T (at most half an ulp of T, one ulp at a binade edge)
plus the error of the kernel's own arithmetic (FP64: a few ulp of the
intermediate sums; FP32: bounded below by 2e-8 for the lattice values here,
|h| < 0.05, up to 19-term sums and a relaxation factor below 2).
"""
import numpy as np

STORES = ("f64", "f32", "f16", "bf16")
MATH_EPS = {"f64": 2e-15, "f32": 2e-8, "f16": 2e-8, "bf16": 2e-8}


def round_to(store, x):
    """Round float64 values to the store format (ties to even), back as float64."""
    x = np.asarray(x, dtype=np.float64)
    if store == "f64":
        return x.copy()
    if store == "f32":
        return x.astype(np.float32).astype(np.float64)
    if store == "f16":
        return x.astype(np.float16).astype(np.float64)
    f = x.astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def ulp(store, x):
    """Spacing of the store format at |x| (subnormal spacing near zero)."""
    x = np.abs(np.asarray(x, dtype=np.float64))
    if store == "f64":
        return np.spacing(x)
    mant, emin = {"f32": (23, -126), "f16": (10, -14), "bf16": (7, -126)}[store]
    e = np.floor(np.log2(np.maximum(x, 2.0 ** emin)))
    return 2.0 ** (e - mant)


def ref_rounding(w, ref):
    """Rounding error of the oracle's own h = f - w: it evaluates f as
    w rho (1 + 3 e.u + ...) with up to four roundings of relative size 2^-53
    in the bracket and one in the product; the subtraction of w is exact."""
    return 6.0 * np.spacing(np.abs(w) + np.abs(ref))


def one_step_tol(store, ref, w=None):
    """ulp of the store at the reference, the arithmetic bound and, when the
    weights are given, the rounding of the reference itself."""
    t = ulp(store, ref) + MATH_EPS[store]
    if w is not None:
        t = t + ref_rounding(w, ref)
    return t


def random_state(orc, shape, store, rng, u_scale=0.05, noise=2e-3):
    """A post-collision state h = f - w, near equilibrium, exactly representable
    in the store format; returned as [19, nz, ny, nx] float64."""
    e, w, _, _ = orc.tables()
    nz, ny, nx = shape
    rho = 1.0 + rng.uniform(-0.02, 0.02, shape)
    u = rng.uniform(-u_scale, u_scale, (3,) + shape)
    u[0] += u_scale
    eu = np.einsum("ai,i...->a...", e.astype(np.float64), u)
    uu = (u * u).sum(axis=0)
    f = w[:, None, None, None] * rho[None] * (1 + 3 * eu + 4.5 * eu * eu - 1.5 * uu[None])
    f = f * (1 + rng.uniform(-noise, noise, f.shape))
    h = (f - w[:, None, None, None]).astype(np.float32).astype(np.float64)
    return round_to(store, h)


def oracle_for(orc, grid, tau, cs, fx, bc, y1=1.0, stats_every=0, collision="bgk", mrt_rates=None, van_driest=0.0,
               van_driest_utau=0.0, wall_nodes=False):
    nx, ny, nz = grid
    bcs = {"bb": orc.BB, "wfb": orc.WFB, "freeslip": orc.FREESLIP}
    p = orc.make_params(nx, ny, nz, tau, cs=cs, fx=fx, bc=bcs[bc], y1=y1, stats_every=stats_every,
                        collision={"bgk": orc.BGK, "mrt": orc.MRT}[collision], rates=mrt_rates,
                        vd_aplus=van_driest, vd_utau=van_driest_utau, wall_nodes=int(wall_nodes))
    return orc.Oracle(p)


def weights(orc):
    return orc.tables()[1][:, None, None, None]
