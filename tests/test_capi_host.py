"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol include/lbmwf.h declares, validates arguments without touching a
device, and its host Spalding inversion agrees with the oracle's."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "lbmwf.h")).read()
    return sorted(set(re.findall(r"^(?:int|void|const char\*|lbm_ctx\*)\s+(lbm_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def L():
    from paper_2009_04352_amd import _lib
    return _lib


def test_exports_every_declared_symbol(L):
    lib = L.lib()
    names = _declared()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.SIGNATURES), "binding and header disagree"


def test_create_validates_arguments(L):
    lib = L.lib()
    h = C.c_void_p()
    bad = [((4, 1, 4), 0.6, 0.1, 0.41, 5.5, 0.0), ((0, 4, 4), 0.6, 0.1, 0.41, 5.5, 0.0),
           ((4, 4, 4), 0.5, 0.1, 0.41, 5.5, 0.0), ((4, 4, 4), float("nan"), 0.1, 0.41, 5.5, 0.0),
           ((4, 4, 4), 0.6, -0.1, 0.41, 5.5, 0.0), ((4, 4, 4), 0.6, 0.1, 0.0, 5.5, 0.0),
           ((4, 4, 4), 0.6, 0.1, 0.41, 5.5, float("inf")), ((2048, 1024, 1024), 0.6, 0.1, 0.41, 5.5, 0.0),
           ((1 << 15, 1 << 14, 1), 0.6, 0.1, 0.41, 5.5, 0.0)]   # a z-plane of 2^29 cells
    for g, *args in bad:
        assert lib.lbm_create(C.byref(L.Grid(*g)), *args, C.byref(h)) == L.LBM_E_ARG
        assert not h.value          # untouched on error
        assert lib.lbm_last_error(None)
    # the largest sizes taken: just below 2^31 cells, and a z-plane just below 2^29
    for g in ((2048, 1023, 1024), ((1 << 28) - 1, 2, 1)):
        assert lib.lbm_create(C.byref(L.Grid(*g)), 0.6, 0.1, 0.41, 5.5, 0.0, C.byref(h)) == L.LBM_OK
        nb = C.c_size_t(0)
        assert lib.lbm_required_bytes(h, C.byref(nb)) == 0 and nb.value == 19 * int(np.prod(g)) * 8
        lib.lbm_destroy(h)
        h = C.c_void_p()
    assert lib.lbm_create(C.byref(L.Grid(4, 4, 4)), 0.6, 0.1, 0.41, 5.5, 1e-6, C.byref(h)) == L.LBM_OK
    try:
        nb = C.c_size_t(0)
        assert lib.lbm_required_bytes(h, C.byref(nb)) == 0 and nb.value == 19 * 64 * 8
        assert lib.lbm_set_param(h, L.LBM_P_STORE, 2) == 0
        assert lib.lbm_required_bytes(h, C.byref(nb)) == 0 and nb.value == 19 * 64 * 2
        assert lib.lbm_set_param(h, L.LBM_P_STORE, 4) == L.LBM_E_ARG
        assert lib.lbm_set_param(h, L.LBM_P_TILE_ODD, 96) == L.LBM_E_ARG
        assert lib.lbm_set_param(h, L.LBM_P_NEWTON_MAXIT, 2.5) == L.LBM_E_ARG
        assert lib.lbm_set_param(h, L.LBM_P_Y1, 0.0) == L.LBM_E_ARG
        assert lib.lbm_set_param(h, L.LBM_P_BC, 1) == L.LBM_E_ARG       # read-only key
        assert lib.lbm_set_boundary(h, 7) == L.LBM_E_ARG
        v = C.c_double()
        assert lib.lbm_get_param(h, L.LBM_P_TAU0, C.byref(v)) == 0 and v.value == 0.6
        # nothing bound yet: stepping or observing is a state error, never a crash
        assert lib.lbm_step(h, 1) == L.LBM_E_STATE
        assert lib.lbm_init_spalding(h, 1e-3, 0.05, 0) == L.LBM_E_STATE
        assert lib.lbm_moments(h, None, None, None, None) == L.LBM_E_STATE
        assert lib.lbm_bind_storage(h, None, 10**6) == L.LBM_E_ARG
        assert lib.lbm_bind_storage(h, C.c_void_p(256), 10) == L.LBM_E_ARG   # too small
        assert b"too small" in lib.lbm_last_error(h)
    finally:
        lib.lbm_destroy(h)


def test_brick_layout_parameter(L):
    """Rows per brick: bricks of 8 rows when every block holds one row, the
    plain layout (one brick of ny rows) when a block holds several."""
    lib = L.lib()
    v = C.c_double()
    for (nx, ny), want in (((512, 128), 8), ((512, 5), 5), ((32, 16), 16)):
        h = C.c_void_p()
        assert lib.lbm_create(C.byref(L.Grid(nx, ny, 4)), 0.6, 0.1, 0.41, 5.5, 0.0, C.byref(h)) == 0
        try:
            assert lib.lbm_get_param(h, L.LBM_P_BRICK, C.byref(v)) == 0 and v.value == want, (nx, ny)
            assert lib.lbm_set_param(h, L.LBM_P_BRICK, 3) == 0
            assert lib.lbm_get_param(h, L.LBM_P_BRICK, C.byref(v)) == 0
            assert v.value == (3 if want != ny or nx >= 256 else ny)
            assert lib.lbm_set_param(h, L.LBM_P_BRICK, -1) == L.LBM_E_ARG
            assert lib.lbm_set_param(h, L.LBM_P_BRICK, 2.5) == L.LBM_E_ARG
        finally:
            lib.lbm_destroy(h)


def test_spread_parameter(L):
    """Brick spreading: chunks of 128 tiles for 2-byte stores and memory order
    otherwise by default; 0 or a chunk log2 in [5, 16]; reads back."""
    lib = L.lib()
    v = C.c_double()
    for store, want in ((L.LBM_STORE_F16, 7), (L.LBM_STORE_F64, 0)):
        h = C.c_void_p()
        assert lib.lbm_create(C.byref(L.Grid(512, 128, 8)), 0.6, 0.1, 0.41, 5.5, 0.0, C.byref(h)) == 0
        try:
            assert lib.lbm_set_param(h, L.LBM_P_STORE, store) == 0
            assert lib.lbm_get_param(h, L.LBM_P_SPREAD, C.byref(v)) == 0 and v.value == want
            for ok in (0, 5, 8, 16):
                assert lib.lbm_set_param(h, L.LBM_P_SPREAD, ok) == 0
                assert lib.lbm_get_param(h, L.LBM_P_SPREAD, C.byref(v)) == 0 and v.value == ok
            for bad in (1, 4, 17, -2, 5.5):
                assert lib.lbm_set_param(h, L.LBM_P_SPREAD, bad) == L.LBM_E_ARG
            assert lib.lbm_set_param(h, L.LBM_P_SPREAD, -1) == 0
            assert lib.lbm_get_param(h, L.LBM_P_SPREAD, C.byref(v)) == 0 and v.value == want
        finally:
            lib.lbm_destroy(h)


def test_odd_kernel_choice_reads_back(L):
    """LBM_P_ODD_BY_ROWS reports the odd kernel the settings select: rows are
    walked for 2-byte and 8-byte stores whose rows are longer than an odd-step
    block (mode 1), always where nx allows (mode 2), never in mode 0; read only."""
    lib = L.lib()
    v = C.c_double()
    cases = [  # nx, store, odd block, mode, walks rows
        (2048, L.LBM_STORE_F16, 128, 1, 1), (512, L.LBM_STORE_F16, 128, 1, 0), (2048, L.LBM_STORE_F64, 256, 1, 1),
        (512, L.LBM_STORE_F64, 512, 1, 0), (2048, L.LBM_STORE_F32, 256, 1, 0), (2048, L.LBM_STORE_F32, 256, 2, 1),
        (2048, L.LBM_STORE_F64, 256, 2, 1), (2048, L.LBM_STORE_F16, 128, 0, 0), (96, L.LBM_STORE_F16, 64, 2, 0)]
    for nx, store, tile, mode, want in cases:
        h = C.c_void_p()
        assert lib.lbm_create(C.byref(L.Grid(nx, 16, 4)), 0.6, 0.1, 0.41, 5.5, 0.0, C.byref(h)) == 0
        try:
            assert lib.lbm_set_param(h, L.LBM_P_STORE, store) == 0
            assert lib.lbm_set_param(h, L.LBM_P_TILE_ODD, tile) == 0
            assert lib.lbm_set_param(h, L.LBM_P_ODD_ROWS, mode) == 0
            assert lib.lbm_get_param(h, L.LBM_P_ODD_BY_ROWS, C.byref(v)) == 0 and v.value == want, (nx, store, mode)
            assert lib.lbm_set_param(h, L.LBM_P_ODD_BY_ROWS, 1) == L.LBM_E_ARG
        finally:
            lib.lbm_destroy(h)


def test_collision_and_damping_parameters(L):
    """Collision 0/1, MRT rates in (0, 2) with the defaults of d'Humieres et
    al. (2002), van Driest A+ and friction velocity >= 0; all read back."""
    lib = L.lib()
    v = C.c_double()
    h = C.c_void_p()
    assert lib.lbm_create(C.byref(L.Grid(64, 16, 4)), 0.6, 0.1, 0.41, 5.5, 1e-6, C.byref(h)) == 0
    try:
        get = lambda k: (lib.lbm_get_param(h, k, C.byref(v)), v.value)[1]
        assert get(L.LBM_P_COLLISION) == L.LBM_BGK
        keys = (L.LBM_P_MRT_S_E, L.LBM_P_MRT_S_EPS, L.LBM_P_MRT_S_Q, L.LBM_P_MRT_S_PI, L.LBM_P_MRT_S_M)
        assert [get(k) for k in keys] == [1.19, 1.4, 1.2, 1.99, 1.98]
        assert get(L.LBM_P_VD_APLUS) == 0.0 and get(L.LBM_P_VD_UTAU) == 0.0
        assert lib.lbm_set_param(h, L.LBM_P_COLLISION, L.LBM_MRT) == 0 and get(L.LBM_P_COLLISION) == L.LBM_MRT
        assert lib.lbm_set_param(h, L.LBM_P_COLLISION, 2) == L.LBM_E_ARG
        for k in keys:
            assert lib.lbm_set_param(h, k, 1.5) == 0 and get(k) == 1.5
            for bad in (0.0, 2.0, -1.0):
                assert lib.lbm_set_param(h, k, bad) == L.LBM_E_ARG
        assert lib.lbm_set_param(h, L.LBM_P_VD_APLUS, 26.0) == 0 and get(L.LBM_P_VD_APLUS) == 26.0
        assert lib.lbm_set_param(h, L.LBM_P_VD_UTAU, 1e-3) == 0 and get(L.LBM_P_VD_UTAU) == 1e-3
        assert lib.lbm_set_param(h, L.LBM_P_VD_APLUS, -1.0) == L.LBM_E_ARG
        assert lib.lbm_set_param(h, L.LBM_P_VD_UTAU, -1.0) == L.LBM_E_ARG
    finally:
        lib.lbm_destroy(h)


def test_status_strings(L):
    lib = L.lib()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert lib.lbm_status_str(code)
    assert lib.lbm_status_str(-99) == b"unknown status"


@pytest.mark.parametrize("yplus", [1e-3, 0.5, 5.0, 11.0, 31.3, 80.0, 640.0, 2003.0, 1e5])
def test_host_spalding_matches_oracle(orc, yplus):
    from paper_2009_04352_amd import spalding_uplus
    up = spalding_uplus(yplus)
    # the oracle evaluates the bracket of Eq. 16 without expm1: ~1e-14 relative at tiny y+
    assert abs(up - orc.spalding_uplus(yplus)) <= 5e-14 * up
    assert abs(orc.spalding_yplus(up) - yplus) <= 1e-12 * yplus


def test_workload_parameters_match_oracle_mapping(orc):
    from paper_2009_04352_amd import workloads as W
    for name, w in W.WORKLOADS.items():
        p = W.params(name)
        q = orc.rule_m(w["grid"][1], w["re_tau"], w["ma"])
        for k in ("u_tau", "nu0", "tau0", "fx", "yplus1"):
            assert abs(p[k] - q[k]) <= 1e-13 * abs(q[k]), (name, k)


def test_wall_node_parameter(L):
    """The wall placement key: 0, 1 or 2, read back; state calls without storage
    are state errors; batches do not take it."""
    lib = L.lib()
    h = C.c_void_p()
    assert lib.lbm_create(C.byref(L.Grid(8, 6, 4)), 0.6, 0.1, 0.41, 5.5, 1e-6, C.byref(h)) == 0
    try:
        v = C.c_double()
        assert lib.lbm_get_param(h, L.LBM_P_WALL_NODES, C.byref(v)) == 0 and v.value == 0.0
        assert lib.lbm_set_param(h, L.LBM_P_WALL_NODES, 0.5) == L.LBM_E_ARG
        assert lib.lbm_set_param(h, L.LBM_P_WALL_NODES, 3) == L.LBM_E_ARG
        assert lib.lbm_set_param(h, L.LBM_P_WALL_NODES, 2) == 0
        assert lib.lbm_get_param(h, L.LBM_P_WALL_NODES, C.byref(v)) == 0 and v.value == 2.0
        assert lib.lbm_set_param(h, L.LBM_P_WALL_NODES, 1) == 0
        assert lib.lbm_get_param(h, L.LBM_P_WALL_NODES, C.byref(v)) == 0 and v.value == 1.0
        fw = np.zeros(10 * 8 * 4)
        assert lib.lbm_get_wall_nodes(h, L.dptr(fw), None) == L.LBM_E_STATE
        assert lib.lbm_moments_device(h, None, None, None, None) == L.LBM_E_STATE
    finally:
        lib.lbm_destroy(h)
    b = C.c_void_p()
    grids = (L.Grid * 1)(L.Grid(8, 6, 4))
    one = np.array([0.6]), np.array([0.1]), np.array([1e-6])
    bc = np.array([1], dtype=np.int32)
    assert lib.lbm_batch_create(1, grids, L.dptr(one[0]), L.dptr(one[1]), L.dptr(one[2]),
                                bc.ctypes.data_as(C.POINTER(C.c_int32)), 0.41, 5.5, C.byref(b)) == 0
    try:
        assert lib.lbm_batch_set_param(b, L.LBM_P_WALL_NODES, 1) == L.LBM_E_ARG
    finally:
        lib.lbm_batch_destroy(b)


def test_yplus_pdf_noalloc_argument_checks(L):
    """The allocation-free y+ distribution checks its arguments before any GPU
    work: null outputs, the bin count, the fixed work area of 2^22 wall cells,
    and a context without storage."""
    lib = L.lib()
    dummy = np.zeros(64)
    p = L.dptr(dummy)
    big = C.c_void_p()
    assert lib.lbm_create(C.byref(L.Grid(2048, 2, 1025)), 0.6, 0.1, 0.41, 5.5, 1e-6, C.byref(big)) == 0
    small = C.c_void_p()
    assert lib.lbm_create(C.byref(L.Grid(2048, 2, 1024)), 0.6, 0.1, 0.41, 5.5, 1e-6, C.byref(small)) == 0
    try:
        assert lib.lbm_wall_yplus_pdf_noalloc(big, 8, -4.0, 4.0, None, p) == L.LBM_E_ARG
        assert lib.lbm_wall_yplus_pdf_noalloc(big, 0, -4.0, 4.0, p, p) == L.LBM_E_ARG
        assert lib.lbm_wall_yplus_pdf_noalloc(big, 8, 4.0, 4.0, p, p) == L.LBM_E_ARG
        assert lib.lbm_wall_yplus_pdf_noalloc(big, 8, -4.0, 4.0, p, p) == L.LBM_E_ARG
        assert b"work area" in lib.lbm_last_error(big)
        # 2 * 2048 * 1024 = 2^22 wall cells fit; without storage the context is not ready
        assert lib.lbm_wall_yplus_pdf_noalloc(small, 8, -4.0, 4.0, p, p) == L.LBM_E_STATE
    finally:
        lib.lbm_destroy(big)
        lib.lbm_destroy(small)


def test_empty_inputs_are_no_ops_or_refused(L):
    """Zero-sized calls that need no device return at once (no device call is
    made, so they run without a GPU); an empty batch is refused."""
    lib = L.lib()
    assert lib.lbm_device_wall_utau(0, None, 1.0, 1e-3, 0.41, 5.5, 1e-14, 50, None, None) == L.LBM_OK
    assert lib.lbm_device_wall_utau(-1, None, 1.0, 1e-3, 0.41, 5.5, 1e-14, 50, None, None) == L.LBM_E_ARG
    assert lib.lbm_codec_roundtrip(2, 0, None, None) == L.LBM_OK
    assert lib.lbm_codec_roundtrip(2, -1, None, None) == L.LBM_E_ARG
    dummy = C.c_void_p(16)   # never dereferenced: zero bytes
    assert lib.lbm_copy_probe(dummy, dummy, 0, None) == L.LBM_OK
    assert lib.lbm_copy_probe(dummy, dummy, 8, None) == L.LBM_E_ARG
    assert lib.lbm_copy_probe(None, dummy, 0, None) == L.LBM_E_ARG
    b = C.c_void_p()
    g = L.Grid(8, 4, 2)
    one = (C.c_double * 1)(0.6)
    bc = (C.c_int32 * 1)(1)
    assert lib.lbm_batch_create(0, C.byref(g), one, one, one, bc, 0.41, 5.5, C.byref(b)) == L.LBM_E_ARG
    assert not b.value


def test_binding_constants_match_the_header(L):
    """Every status code, store, boundary and parameter key of the header has
    the same value in the Python binding."""
    text = open(os.path.join(ROOT, "include", "lbmwf.h")).read()
    defs = re.findall(r"^#define (LBM_(?:P|E|STORE|BB|WFB|FREESLIP|BGK|MRT|OK)\w*)\s+\(?(-?\d+)\)?", text, re.M)
    assert len(defs) > 30
    for name, value in defs:
        assert getattr(L, name) == int(value), name


def test_xcd_chunk_parameter(L):
    """The XCD chunk (log2 of the consecutive tiles each XCD takes in turn) is
    an integer in [0, 12], default 5; batches keep theirs."""
    lib = L.lib()
    h = C.c_void_p()
    assert lib.lbm_create(C.byref(L.Grid(64, 6, 4)), 0.6, 0.1, 0.41, 5.5, 0.0, C.byref(h)) == 0
    try:
        v = C.c_double()
        assert lib.lbm_get_param(h, L.LBM_P_XCD_CHUNK, C.byref(v)) == 0 and v.value == 5.0
        for ok in (0, 7, 12):
            assert lib.lbm_set_param(h, L.LBM_P_XCD_CHUNK, ok) == 0
            assert lib.lbm_get_param(h, L.LBM_P_XCD_CHUNK, C.byref(v)) == 0 and v.value == ok
        for bad in (-1, 13, 2.5):
            assert lib.lbm_set_param(h, L.LBM_P_XCD_CHUNK, bad) == L.LBM_E_ARG
    finally:
        lib.lbm_destroy(h)
    b = C.c_void_p()
    g = (L.Grid * 1)(L.Grid(8, 4, 2))
    one = (C.c_double * 1)(0.6)
    bc = (C.c_int32 * 1)(1)
    assert lib.lbm_batch_create(1, g, one, one, one, bc, 0.41, 5.5, C.byref(b)) == 0
    try:
        assert lib.lbm_batch_set_param(b, L.LBM_P_XCD_CHUNK, 7) == L.LBM_E_ARG
    finally:
        lib.lbm_batch_destroy(b)
