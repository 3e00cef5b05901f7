"""The channel workloads measured and parity-tested, as seeded synthetic inputs.

Every workload is the paper's channel (Sec. 3.1: x streamwise and periodic, y
wall-normal with walls at both ends, z spanwise and periodic, D = ny / 2) with
Smagorinsky Cs = 0.1 and Spalding constants kappa = 0.41, B = 5.5 (Eq. 16),
started from the Spalding profile with 5 % seeded uniform noise.  Lattice
parameters follow the low-Mach mapping of Table 1: the centreline speed is
Ma_LB * c_s, u_tau = u_c / u+(Re_tau), nu0 = u_tau D / Re_tau,
tau0 = 1/2 + 3 nu0, Fx = u_tau^2 / D.  A workload may instead name tau
directly, keeping u_tau and Fx.

No workload reads a dataset: the paper's inputs are the geometry and these
parameters, not data.
"""
import math

from .channel import spalding_uplus

KAPPA, B, CS = 0.41, 5.5, 0.1


def rule_m(ny, re_tau, ma, y1=1.0, kappa=KAPPA, b=B):
    D = ny / 2.0
    uc = ma / math.sqrt(3.0)
    u_tau = uc / spalding_uplus(re_tau, kappa, b)
    nu0 = u_tau * D / re_tau
    return dict(u_tau=u_tau, nu0=nu0, tau0=0.5 + 3.0 * nu0, fx=u_tau * u_tau / D, yplus1=y1 * u_tau / nu0)


# name: grid, Re_tau, Ma_LB (Table 1), steps, stores, boundaries, named tau (or None)
WORKLOADS = {
    "c1": dict(grid=(32, 16, 16), re_tau=640.0, ma=0.060, steps=200, stores=("f64",), bcs=("wfb", "bb"),
               tau=0.51, desc="plain FP64 single channel 32x16x16, Re_tau 640, 200 steps"),
    "c2": dict(grid=(128, 64, 64), re_tau=640.0, ma=0.060, steps=10000, stores=("f32",), bcs=("wfb", "bb"),
               tau=None, stats_every=1, desc="single channel 128x64x64, Re_tau 640, FP32, 10k steps, FP64 plane statistics"),
    "c3": dict(grid=(512, 128, 256), re_tau=2003.0, ma=0.069, steps=2000, stores=("f64", "f32", "f16", "bf16"),
               bcs=("wfb",), tau=0.503, desc="single channel 512x128x256 (16.8M cells), Re_tau 2003, WFB, 2k steps"),
    "c5": dict(grid=(2048, 512, 1024), re_tau=2003.0, ma=0.069, steps=500, stores=("f16", "f32"), bcs=("wfb",),
               tau=None, desc="large channel 2048x512x1024 (1.07B cells), Re_tau 2003, WFB, 500 steps"),
    # one GPU's share of c5 split into 8 x-slabs, at its real shape (periodic
    # in x here: the halo exchange of a multi-GPU run is not built)
    "c5s": dict(grid=(256, 512, 1024), re_tau=2003.0, ma=0.069, steps=500, stores=("f64", "f32", "f16", "bf16"),
                bcs=("wfb",), tau=None,
                desc="one GPU's x-slab of the 2048x512x1024 channel over 8 GPUs, 256x512x1024 (134M cells), "
                     "Re_tau 2003, WFB, 500 steps"),
}

# The paper's own cases (Table 1): grid, Re_tau, Ma_LB; used by the wall-law
# validation runs, not by the benchmark.
TABLE1 = {
    "A20": dict(grid=(128, 40, 64), re_tau=640.0, ma=0.060, tau=None),
    "A40": dict(grid=(256, 80, 128), re_tau=640.0, ma=0.060, tau=None),
    "B40": dict(grid=(256, 80, 128), re_tau=2003.0, ma=0.069, tau=None),
    "B80": dict(grid=(512, 160, 256), re_tau=2003.0, ma=0.069, tau=None),
}


def case(name):
    """The workload or Table 1 case of that name."""
    return WORKLOADS[name] if name in WORKLOADS else TABLE1[name]


# the batched ensemble (see ensemble()): 64 channels, FP32 store, 1000 steps
ENSEMBLE = dict(n=64, store="f32", steps=1000,
                desc="64 independent channels, grids {32,64,128}x{16,32,64}x{16,32,64}, Re_tau in [300,2003), "
                     "half WFB half BB, FP32, one launch per step")


def splitmix64(seed, k):
    """Output k of splitmix64 (Steele, Lea & Flood 2014) from state `seed`:
    the draws of the ensemble recipe below."""
    m = (1 << 64) - 1
    z = (seed + (k + 1) * 0x9E3779B97F4A7C15) & m
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
    return z ^ (z >> 31)


def ensemble(n=64, ma=0.060):
    """The batched ensemble: instance i (seed i) draws nx from {32, 64, 128},
    ny and nz from {16, 32, 64} and Re_tau uniformly in [300, 2003) by
    splitmix64 of state i; WFB walls for even i, bounce-back for odd i.
    Returns one dict per instance (grid, lattice parameters, boundary)."""
    out = []
    for i in range(n):
        u = [splitmix64(i, k) for k in range(4)]
        nx = (32, 64, 128)[u[0] % 3]
        ny = (16, 32, 64)[u[1] % 3]
        nz = (16, 32, 64)[u[2] % 3]
        re_tau = 300.0 + 1703.0 * ((u[3] >> 11) * (1.0 / 9007199254740992.0))
        p = rule_m(ny, re_tau, ma)
        out.append(dict(nx=nx, ny=ny, nz=nz, re_tau=re_tau, tau=p["tau0"], cs=CS, fx=p["fx"], u_tau=p["u_tau"],
                        bc="wfb" if i % 2 == 0 else "bb", seed=i))
    return out


def params(name, named_tau=False):
    """Lattice parameters of a workload: dict(grid, tau0, fx, u_tau, ...)."""
    w = case(name)
    nx, ny, nz = w["grid"]
    p = rule_m(ny, w["re_tau"], w["ma"])
    if named_tau:
        if w["tau"] is None:
            raise ValueError("workload %s names no tau" % name)
        p["tau0"] = w["tau"]
        p["nu0"] = (w["tau"] - 0.5) / 3.0
        p["yplus1"] = p["u_tau"] / p["nu0"]
    p.update(grid=(nx, ny, nz), cs=CS, kappa=KAPPA, B=B, noise=0.05, seed=0)
    return p


# Launch shapes used by the benchmark and by the full-size parity tests, per
# workload and store format: (threads per block of the odd kernel, of the even
# kernel, cells per thread), measured on MI355X.  FP64 and FP32 run one cell
# per thread: in row segments their odd step shifts by plain address offsets
# (FP32 on the 512 x 128 x 256 channel: 128-thread odd segments, whole-row
# even blocks; on the 2,048-cell rows of the large channel 512- and 256-cell
# segments), on whole rows through LDS (FP64 on 512-cell rows).  FP16/BF16 run
# four cells per thread (8-byte groups); their odd step walks rows one
# wavefront each on the large channel, whose even step runs 4 % faster in
# blocks of 256 threads than of 128.  The benchmark's autotuner starts from
# this table.
LAUNCH_TILES = {
    "c2": {"f64": (128, 128, 1), "f32": (64, 64, 2), "f16": (64, 64, 2), "bf16": (64, 64, 2)},
    "c3": {"f64": (512, 512, 1), "f32": (128, 256, 1), "f16": (128, 128, 4), "bf16": (128, 128, 4)},
    "c5": {"f64": (512, 256, 1), "f32": (256, 256, 1), "f16": (128, 256, 4), "bf16": (128, 256, 4)},
    "c5s": {"f64": (256, 256, 1), "f32": (256, 256, 1), "f16": (64, 64, 4), "bf16": (64, 64, 4)},
}
# With the MRT collision the 2-byte odd step needs more registers than three
# wavefronts per SIMD allow at 4 cells per thread; at 2 cells per thread it
# keeps three, and the pair of steps runs 5-6 % faster on the 512-cell rows.
# On the 2048-cell rows the odd step walks rows at 2 cells per thread (21.5 ms
# against 23.4 ms at 4 cells per thread in FP16, 32.5 ms in BF16).
LAUNCH_TILES_MRT = {"c3": {"f16": (256, 256, 2), "bf16": (256, 256, 2)},
                    "c5": {"f16": (64, 128, 2), "bf16": (64, 256, 2)}}


def launch_tiles(workload, store, collision="bgk"):
    if collision == "mrt" and store in LAUNCH_TILES_MRT.get(workload, {}):
        return LAUNCH_TILES_MRT[workload][store]
    return LAUNCH_TILES.get(workload, LAUNCH_TILES["c3"])[store]


def sample_cells(grid, n, seed=0):
    """Cell indices for sampled full-size checks: every corner and edge cell of
    the wall rows' periodic seams plus n uniformly drawn cells."""
    import numpy as np
    nx, ny, nz = grid
    rng = np.random.default_rng(seed)
    xs = np.array([0, 1, nx - 2, nx - 1])
    ys = np.array([0, 1, ny - 2, ny - 1])
    zs = np.array([0, 1, nz - 2, nz - 1])
    X, Y, Z = np.meshgrid(xs, ys, zs, indexing="ij")
    seam = (X + nx * (Y + ny * Z)).ravel()
    rand = rng.integers(0, nx * ny * nz, n)
    return np.unique(np.concatenate([seam, rand])).astype(np.int64)
