"""Python face of the C ABI: one channel context on one GPU.

PyTorch provides the device memory (a uint8 tensor the library binds) and
the stream; every step of the computation runs in the library's HIP kernels.
"""
import ctypes as C

import numpy as np

from . import _lib as L

STORES = {"f64": L.LBM_STORE_F64, "f32": L.LBM_STORE_F32, "f16": L.LBM_STORE_F16, "bf16": L.LBM_STORE_BF16}
BOUNDARIES = {"bb": L.LBM_BB, "wfb": L.LBM_WFB, "freeslip": L.LBM_FREESLIP}


MRT_KEYS = {"s_e": L.LBM_P_MRT_S_E, "s_eps": L.LBM_P_MRT_S_EPS, "s_q": L.LBM_P_MRT_S_Q,
            "s_pi": L.LBM_P_MRT_S_PI, "s_m": L.LBM_P_MRT_S_M}


def set_collision(setter, collision="bgk", mrt_rates=None, van_driest=0.0, van_driest_utau=0.0):
    """Collision operator ("bgk" or "mrt"), MRT rates by name (s_e, s_eps,
    s_q, s_pi, s_m; others keep their defaults) and the van Driest A+ (0: off)
    with the friction velocity of its y+ (0: from the force balance)."""
    setter(L.LBM_P_COLLISION, {"bgk": L.LBM_BGK, "mrt": L.LBM_MRT}[collision])
    for k, v in (mrt_rates or {}).items():
        setter(MRT_KEYS[k], v)
    setter(L.LBM_P_VD_APLUS, van_driest)
    setter(L.LBM_P_VD_UTAU, van_driest_utau)


def spalding_uplus(yplus, kappa=0.41, B=5.5):
    """u+ of Spalding's law at y+ (host inversion in the library)."""
    out = C.c_double(0.0)
    L.check(L.lib().lbm_spalding_uplus(float(yplus), float(kappa), float(B), C.byref(out)))
    return out.value


def device_wall_utau(U, y1, nu, kappa=0.41, B=5.5, tol=1e-14, maxit=100):
    """The step kernel's FP64 wall-function solve on the GPU for each speed in U:
    returns (u_tau, iterations); u_tau = -1 marks an iteration-cap failure."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    ut = np.zeros_like(U)
    it = np.zeros(U.shape, dtype=np.int32)
    L.check(L.lib().lbm_device_wall_utau(U.size, L.dptr(U), y1, nu, kappa, B, tol, maxit, L.dptr(ut),
                                         it.ctypes.data_as(C.POINTER(C.c_int32))))
    return ut, it


def codec_roundtrip(store, values):
    """decode(encode(v)) through the store format's device codec (float32 in and out)."""
    v = np.ascontiguousarray(values, dtype=np.float32)
    out = np.empty_like(v)
    fp = C.POINTER(C.c_float)
    L.check(L.lib().lbm_codec_roundtrip(STORES[store], v.size, v.ctypes.data_as(fp), out.ctypes.data_as(fp)))
    return out


def copy_probe(dst, src, nbytes, stream=None):
    """Plain device copy of nbytes (multiple of 16) between two torch tensors."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    L.check(L.lib().lbm_copy_probe(C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()), int(nbytes),
                                   C.c_void_p(s.cuda_stream)))


class Channel:
    """A D3Q19 channel (x, z periodic, walls in y) advanced on the GPU."""

    def __init__(self, nx, ny, nz, tau, cs=0.1, kappa=0.41, B=5.5, fx=0.0, store="f64", bc="wfb", y1=1.0,
                 device="cuda", stream=None, tiles=None, graph_steps=None, stats_every=0, autotune=False,
                 vector=0, brick=0, collision="bgk", mrt_rates=None, van_driest=0.0, van_driest_utau=0.0,
                 wall_nodes=False, storage=None):
        """storage: an optional contiguous uint8 torch tensor on the device to bind
        instead of a fresh allocation (at least the required bytes; its data
        pointer 256-byte aligned), e.g. one buffer shared by channels run one
        after the other."""
        import torch
        self.lib = L.lib()
        self.shape = (nz, ny, nx)
        self.nx, self.ny, self.nz = nx, ny, nz
        self.ncell = nx * ny * nz
        self.store = store
        h = C.c_void_p()
        L.check(self.lib.lbm_create(C.byref(L.Grid(nx, ny, nz)), tau, cs, kappa, B, fx, C.byref(h)))
        self._h = h
        self._set(L.LBM_P_STORE, STORES[store])
        self._set(L.LBM_P_Y1, y1)
        if stats_every:
            self._set(L.LBM_P_STATS_EVERY, stats_every)
        if graph_steps is not None:
            self._set(L.LBM_P_GRAPH_STEPS, graph_steps)
        if tiles is not None:
            self._set(L.LBM_P_TILE_ODD, tiles[0])
            self._set(L.LBM_P_TILE_EVEN, tiles[1])
            if len(tiles) > 2:
                vector = tiles[2]
        if vector:
            self._set(L.LBM_P_VECTOR, vector)
        if brick:
            self._set(L.LBM_P_BRICK, brick)
        set_collision(self._set, collision, mrt_rates, van_driest, van_driest_utau)
        if wall_nodes:
            self._set(L.LBM_P_WALL_NODES, int(wall_nodes))   # True / 1: stress of the previous step; 2: same step
        nbytes = C.c_size_t(0)
        L.check(self.lib.lbm_required_bytes(self._h, C.byref(nbytes)), self._h)
        self.nbytes = nbytes.value
        self.device = torch.device(device)
        if storage is None:
            self.storage = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        else:
            if storage.dtype != torch.uint8 or not storage.is_contiguous() or storage.numel() < self.nbytes:
                raise ValueError("storage must be a contiguous uint8 tensor of at least %d bytes" % self.nbytes)
            self.storage = storage
            self.device = storage.device
        L.check(self.lib.lbm_bind_storage(self._h, C.c_void_p(self.storage.data_ptr()), self.nbytes), self._h)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        L.check(self.lib.lbm_set_stream(self._h, C.c_void_p(self.stream.cuda_stream)), self._h)
        self.set_boundary(bc)
        self.tiles = None
        if autotune:
            self.autotune()

    # -- plumbing
    def _chk(self, code):
        return L.check(code, self._h)

    def _set(self, key, value):
        self._chk(self.lib.lbm_set_param(self._h, key, float(value)))

    def get_param(self, key):
        v = C.c_double(0.0)
        self._chk(self.lib.lbm_get_param(self._h, key, C.byref(v)))
        return v.value

    def set_param(self, key, value):
        self._set(key, value)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.lbm_destroy(self._h)
            self._h = C.c_void_p()
        self.storage = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- set-up
    def set_boundary(self, bc):
        self._chk(self.lib.lbm_set_boundary(self._h, BOUNDARIES[bc] if isinstance(bc, str) else int(bc)))

    def autotune(self, steps=6):
        """Tunes the launch shapes from the current ones (lbm_autotune); returns
        a dict: tile_odd, tile_even, vector (cells per thread), brick (rows per
        brick in use), spread (launch-order chunk log2, 0 = memory order),
        odd_rows (1 if the odd step walks rows), cached (1 if taken from the
        process's cache of earlier results for this grid, store and boundary),
        xcd_chunk (log2 of the consecutive tiles each XCD takes in turn)."""
        t = (C.c_int32 * 8)()
        self._chk(self.lib.lbm_autotune(self._h, int(steps), t))
        keys = ("tile_odd", "tile_even", "vector", "brick", "spread", "odd_rows", "cached", "xcd_chunk")
        self.tiles = (t[0], t[1], t[2])
        return dict(zip(keys, list(t)))

    def init_spalding(self, u_tau, noise=0.05, seed=0):
        self._chk(self.lib.lbm_init_spalding(self._h, float(u_tau), float(noise), int(seed)))

    def init_moments(self, rho, u):
        """f = f_eq(rho, u) as the post-collision state of step 0; rho is
        [nz, ny, nx] (or flat), u is [3, nz, ny, nx] (or [3, ncell])."""
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
        if rho.size != self.ncell or u.size != 3 * self.ncell:
            raise ValueError("rho must hold ncell values and u 3 * ncell")
        self._chk(self.lib.lbm_init_moments(self._h, L.dptr(rho), L.dptr(u)))

    def set_state(self, h, steps=0):
        """h: [19, nz, ny, nx] (or flat) float64, post-collision f - w."""
        h = np.ascontiguousarray(h, dtype=np.float64).reshape(-1)
        if h.size != 19 * self.ncell:
            raise ValueError("state must hold 19 * ncell values")
        self._chk(self.lib.lbm_set_state(self._h, L.dptr(h), int(steps)))

    def get_state(self):
        out = np.empty(19 * self.ncell)
        self._chk(self.lib.lbm_get_state(self._h, L.dptr(out)))
        return out.reshape((19,) + self.shape)

    def get_state_cells(self, cells):
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        out = np.empty(19 * len(cells))
        self._chk(self.lib.lbm_get_state_cells(self._h, len(cells), L.i64ptr(cells), L.dptr(out)))
        return out.reshape(19, len(cells)).T.copy()

    # -- time stepping
    def step(self, n=1):
        self._chk(self.lib.lbm_step(self._h, int(n)))

    def sync(self):
        """Returns (status, first bad step); raises nothing."""
        fb = C.c_int64(-1)
        st = self.lib.lbm_sync(self._h, C.byref(fb))
        return st, fb.value

    @property
    def steps(self):
        s = C.c_int64(0)
        self._chk(self.lib.lbm_steps_done(self._h, C.byref(s)))
        return s.value

    # -- observation
    def moments(self):
        outs = [np.empty(self.ncell) for _ in range(4)]
        self._chk(self.lib.lbm_moments(self._h, *[L.dptr(o) for o in outs]))
        return tuple(o.reshape(self.shape) for o in outs)

    def moments_cells(self, cells):
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        out = np.empty(4 * len(cells))
        self._chk(self.lib.lbm_moments_cells(self._h, len(cells), L.i64ptr(cells), L.dptr(out)))
        return out.reshape(len(cells), 4)

    def moments_device(self, rho=None, ux=None, uy=None, uz=None):
        """Observables written into float64 torch tensors of ncell elements on the
        channel's device (any may be None), enqueued on the channel's stream."""
        ptrs = []
        for t in (rho, ux, uy, uz):
            if t is None:
                ptrs.append(None)
                continue
            import torch
            if t.dtype != torch.float64 or t.numel() < self.ncell or not t.is_contiguous():
                raise ValueError("moment tensors must be contiguous float64 with ncell elements")
            ptrs.append(C.c_void_p(t.data_ptr()))
        self._chk(self.lib.lbm_moments_device(self._h, *ptrs))

    def wall_shear(self):
        m = 2 * self.nx * self.nz
        outs = [np.empty(m) for _ in range(4)]
        self._chk(self.lib.lbm_wall_shear(self._h, *[L.dptr(o) for o in outs]))
        return tuple(o.reshape(2, self.nz, self.nx) for o in outs)

    def wall_yplus_pdf(self, nbins=40, lo=-4.0, hi=4.0):
        """Distribution of the first-layer y+ normalised by its mean and standard
        deviation (Fig. 7): returns (counts[nbins + 2] with under- and overflow
        bins first and last, bin edges, mean, std)."""
        counts = np.zeros(nbins + 2, dtype=np.int64)
        ms = np.zeros(2)
        self._chk(self.lib.lbm_wall_yplus_pdf(self._h, nbins, lo, hi, counts.ctypes.data_as(C.c_void_p),
                                              L.dptr(ms)))
        return counts, np.linspace(lo, hi, nbins + 1), ms[0], ms[1]

    def wall_yplus_pdf_noalloc(self, counts, mean_std, nbins=40, lo=-4.0, hi=4.0):
        """wall_yplus_pdf into caller-owned device tensors (int64 counts of
        nbins + 2 elements, float64 mean_std of 2), enqueued on the channel's
        stream with no allocation by the library."""
        import torch
        if (counts.dtype != torch.int64 or counts.numel() < nbins + 2 or not counts.is_contiguous()
                or mean_std.dtype != torch.float64 or mean_std.numel() < 2 or not mean_std.is_contiguous()):
            raise ValueError("counts: contiguous int64 of nbins + 2; mean_std: contiguous float64 of 2")
        self._chk(self.lib.lbm_wall_yplus_pdf_noalloc(self._h, nbins, lo, hi, C.c_void_p(counts.data_ptr()),
                                                      C.c_void_p(mean_std.data_ptr())))

    def wall_mass_change(self):
        """Eq. B-1 per wall cell: (change of the population sum made by the WFB
        correction the next step would apply, density before it), each of
        shape (2, nz, nx), bottom wall first."""
        ds = np.empty(2 * self.nx * self.nz)
        rho = np.empty(2 * self.nx * self.nz)
        self._chk(self.lib.lbm_wall_mass_change(self._h, L.dptr(ds), L.dptr(rho)))
        return ds.reshape(2, self.nz, self.nx), rho.reshape(2, self.nz, self.nx)

    def wall_nodes(self):
        """Wall-node state: (fw [2, 5, nz, nx] as h = f - w, what the wall nodes send
        into the fluid next step; rec [2, nz, nx, 4]: the first layer's rho, u_x,
        u_z, u_tau of the latest step)."""
        fw = np.empty(10 * self.nx * self.nz)
        rec = np.empty(8 * self.nx * self.nz)
        self._chk(self.lib.lbm_get_wall_nodes(self._h, L.dptr(fw), L.dptr(rec)))
        return fw.reshape(2, 5, self.nz, self.nx), rec.reshape(2, self.nz, self.nx, 4)

    def stats_reset(self):
        self._chk(self.lib.lbm_stats_reset(self._h))

    def stats_sums(self):
        out = np.empty(8 * self.ny)
        ns = C.c_int64(0)
        self._chk(self.lib.lbm_stats_sums(self._h, L.dptr(out), C.byref(ns)))
        return out.reshape(self.ny, 8), ns.value

    def stats(self):
        out = np.empty(8 * self.ny)
        ns = C.c_int64(0)
        self._chk(self.lib.lbm_stats_get(self._h, L.dptr(out), C.byref(ns)))
        return out.reshape(self.ny, 8), ns.value


class _InstanceView(Channel):
    """Observation handle on one instance of a Batch (owned by the batch)."""

    def __init__(self, batch, i, nx, ny, nz, store):
        self.lib = L.lib()
        self.shape = (nz, ny, nx)
        self.nx, self.ny, self.nz = nx, ny, nz
        self.ncell = nx * ny * nz
        self.store = store
        self._h = C.c_void_p(self.lib.lbm_batch_instance(batch._h, i))
        self._batch = batch  # keeps the batch (and its storage) alive

    def close(self):
        self._h = C.c_void_p()


class Batch:
    """Independent channels advanced together: one launch per step over the
    tiles of every instance.  specs: list of dicts with keys nx, ny, nz, tau,
    cs, fx, bc."""

    def __init__(self, specs, kappa=0.41, B=5.5, store="f32", device="cuda", stream=None, tiles=None,
                 graph_steps=None, vector=0, brick=0, collision="bgk", mrt_rates=None, van_driest=0.0,
                 van_driest_utau=0.0):
        import torch
        self.lib = L.lib()
        n = len(specs)
        grids = (L.Grid * n)(*[L.Grid(s["nx"], s["ny"], s["nz"]) for s in specs])
        arr = lambda k: np.ascontiguousarray([float(s[k]) for s in specs])
        self._tau, self._cs, self._fx = arr("tau"), arr("cs"), arr("fx")
        bcs = np.ascontiguousarray([BOUNDARIES[s["bc"]] if isinstance(s["bc"], str) else int(s["bc"]) for s in specs],
                                   dtype=np.int32)
        h = C.c_void_p()
        L.check_batch(self.lib.lbm_batch_create(n, grids, L.dptr(self._tau), L.dptr(self._cs), L.dptr(self._fx),
                                                bcs.ctypes.data_as(C.POINTER(C.c_int32)), kappa, B, C.byref(h)))
        self._h = h
        self.specs = specs
        self.n = n
        self.store = store
        self._set(L.LBM_P_STORE, STORES[store])
        if graph_steps is not None:
            self._set(L.LBM_P_GRAPH_STEPS, graph_steps)
        if tiles is not None:
            self._set(L.LBM_P_TILE_ODD, tiles[0])
            self._set(L.LBM_P_TILE_EVEN, tiles[1])
            if len(tiles) > 2:
                vector = tiles[2]
        if vector:
            self._set(L.LBM_P_VECTOR, vector)
        if brick:
            self._set(L.LBM_P_BRICK, brick)
        set_collision(self._set, collision, mrt_rates, van_driest, van_driest_utau)
        nbytes = C.c_size_t(0)
        L.check_batch(self.lib.lbm_batch_required_bytes(self._h, C.byref(nbytes)), self._h)
        self.nbytes = nbytes.value
        self.device = torch.device(device)
        self.storage = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        L.check_batch(self.lib.lbm_batch_bind_storage(self._h, C.c_void_p(self.storage.data_ptr()), self.nbytes),
                      self._h)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        L.check_batch(self.lib.lbm_batch_set_stream(self._h, C.c_void_p(self.stream.cuda_stream)), self._h)
        self.ncell = sum(s["nx"] * s["ny"] * s["nz"] for s in specs)

    def _set(self, key, value):
        L.check_batch(self.lib.lbm_batch_set_param(self._h, key, float(value)), self._h)

    def autotune(self, steps=6):
        t = (C.c_int32 * 3)()
        L.check_batch(self.lib.lbm_batch_autotune(self._h, int(steps), t), self._h)
        return (t[0], t[1], t[2])

    def init_spalding(self, u_tau, noise=0.05, seeds=None):
        ut = np.ascontiguousarray(u_tau, dtype=np.float64)
        sd = np.ascontiguousarray(seeds if seeds is not None else np.arange(self.n), dtype=np.uint64)
        L.check_batch(self.lib.lbm_batch_init_spalding(self._h, L.dptr(ut), float(noise),
                                                       sd.ctypes.data_as(C.POINTER(C.c_uint64))), self._h)

    def step(self, n=1):
        L.check_batch(self.lib.lbm_batch_step(self._h, int(n)), self._h)

    def sync(self):
        """Returns (status, first bad step, first bad instance)."""
        fb, fi = C.c_int64(-1), C.c_int32(-1)
        st = self.lib.lbm_batch_sync(self._h, C.byref(fb), C.byref(fi))
        return st, fb.value, fi.value

    def instance(self, i):
        s = self.specs[i]
        return _InstanceView(self, i, s["nx"], s["ny"], s["nz"], self.store)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.lbm_batch_destroy(self._h)
            self._h = C.c_void_p()
        self.storage = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
