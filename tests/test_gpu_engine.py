"""GPU checks of the launch machinery: graph replay equals eager launches,
results do not depend on the block size or the XCD remap, checkpoint/resume
is exact, and device-side failures surface with their step."""
import numpy as np
import pytest

from gpu_common import random_state, weights

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_04352_amd as P
    return P


def _state(orc, grid, store, seed):
    return random_state(orc, grid[::-1], store, np.random.default_rng(seed))


@pytest.mark.parametrize("store", ("f64", "f32", "f16"))
def test_graph_replay_equals_eager(P, orc, store):
    grid = (130, 6, 5)
    h0 = _state(orc, grid, store, 1)
    out = []
    for gs in (0, 8, 5):
        ch = P.Channel(*grid, 0.51, cs=0.1, fx=1e-6, store=store, bc="wfb", graph_steps=gs, stats_every=3)
        ch.set_state(h0)
        for n in (3, 17, 8):       # chunks that start at both parities and stats phases
            ch.step(n)
        out.append((ch.get_state(), ch.stats_sums()[0]))
    for s, st in out[1:]:
        assert np.array_equal(s, out[0][0])
        assert np.array_equal(st, out[0][1])


@pytest.mark.parametrize("store", ("f64", "f32", "bf16"))
def test_block_size_and_remap_invariance(P, orc, store):
    grid = (200, 7, 6)
    h0 = _state(orc, grid, store, 2)
    ref = None
    from paper_2009_04352_amd import _lib as L
    for tiles in ((64, 64), (128, 256), (256, 512), (512, 128)):
        for remap, chunk in ((0, 5), (1, 5), (1, 0), (1, 2), (1, 9)):
            ch = P.Channel(*grid, 0.505, cs=0.1, fx=1e-6, store=store, bc="wfb", tiles=tiles)
            ch.set_param(L.LBM_P_XCD_REMAP, remap)
            ch.set_param(L.LBM_P_XCD_CHUNK, chunk)
            ch.set_state(h0)
            ch.step(9)
            s = ch.get_state()
            if ref is None:
                ref = s
            assert np.array_equal(s, ref), (tiles, remap, chunk)


def test_autotune_picks_valid_shapes_and_caches_them(P):
    """The tuner's choice is a valid set of launch shapes that the context
    reads back, a second context of the same grid, store and boundary gets it
    from the cache, and the tuned shapes give the default shapes' bits."""
    from paper_2009_04352_amd import _lib as L
    grid = (256, 24, 16)
    ch = P.Channel(*grid, 0.51, fx=1e-6, store="f32", bc="wfb")
    t = ch.autotune(steps=4)
    assert t["cached"] == 0
    assert t["tile_odd"] in (64, 128, 256, 512) and t["tile_even"] in (64, 128, 256, 512)
    assert t["vector"] in (1, 2) and t["spread"] in (0, 5, 7, 9) and t["odd_rows"] in (0, 1)
    assert 1 <= t["brick"] <= grid[1] and t["xcd_chunk"] in (5, 7, 9)
    for key, name in ((L.LBM_P_TILE_ODD, "tile_odd"), (L.LBM_P_TILE_EVEN, "tile_even"), (L.LBM_P_VECTOR, "vector"),
                      (L.LBM_P_BRICK, "brick"), (L.LBM_P_SPREAD, "spread"), (L.LBM_P_ODD_BY_ROWS, "odd_rows"),
                      (L.LBM_P_XCD_CHUNK, "xcd_chunk")):
        assert ch.get_param(key) == t[name], name
    again = P.Channel(*grid, 0.51, fx=1e-6, store="f32", bc="wfb")
    t2 = again.autotune(steps=4)
    assert t2["cached"] == 1 and {k: v for k, v in t2.items() if k != "cached"} == \
        {k: v for k, v in t.items() if k != "cached"}
    plain = P.Channel(*grid, 0.51, fx=1e-6, store="f32", bc="wfb")
    for c in (ch, plain):
        c.init_spalding(0.01, 0.05, 3)
        c.step(9)
        assert c.sync()[0] == 0
    np.testing.assert_array_equal(ch.get_state(), plain.get_state())
    with pytest.raises(P.LbmError):
        ch.autotune()           # only before the state is initialised
    for c in (ch, again, plain):
        c.close()


@pytest.mark.parametrize("k", (3, 4))
def test_checkpoint_resume_is_exact(P, orc, k):
    grid = (67, 5, 4)
    h0 = _state(orc, grid, "f32", 5)
    a = P.Channel(*grid, 0.51, cs=0.1, fx=1e-6, store="f32", bc="wfb")
    a.set_state(h0)
    a.step(10)
    ref = a.get_state()
    b = P.Channel(*grid, 0.51, cs=0.1, fx=1e-6, store="f32", bc="wfb")
    b.set_state(h0)
    b.step(k)
    saved, steps = b.get_state(), b.steps
    c = P.Channel(*grid, 0.51, cs=0.1, fx=1e-6, store="f32", bc="wfb")
    c.set_state(saved, steps=steps)
    c.step(10 - k)
    assert c.steps == 10
    assert np.array_equal(c.get_state(), ref)


def test_nonfinite_is_reported_with_its_step(P, orc):
    grid = (64, 4, 4)
    h0 = _state(orc, grid, "f64", 6)
    h0[5, 2, 1, 7] = np.nan
    ch = P.Channel(*grid, 0.52, fx=0.0, store="f64", bc="bb")
    ch.set_state(h0, steps=40)
    ch.step(3)
    st, first = ch.sync()
    assert st == -5 and first == 41
    with pytest.raises(P.LbmError):
        ch.moments()


def test_newton_cap_is_reported(P, orc):
    grid = (64, 4, 4)
    ch = P.Channel(*grid, 0.50001, cs=0.0, fx=0.0, store="f64", bc="wfb")
    ch.set_param(2, 1)            # one Newton iteration cannot converge
    h0 = _state(orc, grid, "f64", 7)
    ch.set_state(h0)
    ch.step(1)
    st, first = ch.sync()
    assert st == -6 and first == 1


def test_argument_errors_do_not_touch_outputs(P):
    ch = P.Channel(8, 4, 4, 0.6, store="f32")
    with pytest.raises(P.LbmError):
        ch.step(1)                 # not initialised
    ch.init_spalding(1e-3)
    out = np.full(19 * 2, 7.0)
    import ctypes as C
    from paper_2009_04352_amd import _lib as L
    bad = np.array([0, 10**6], dtype=np.int64)
    st = L.lib().lbm_get_state_cells(ch._h, 2, L.i64ptr(bad), L.dptr(out))
    assert st == L.LBM_E_ARG and np.all(out == 7.0)
    assert L.lib().lbm_step(ch._h, -1) == L.LBM_E_ARG
    assert L.lib().lbm_set_param(ch._h, L.LBM_P_STORE, 0) == L.LBM_E_STATE
    assert C is not None


@pytest.mark.parametrize("store", ("f64", "f16"))
def test_brick_layout_invariance(P, orc, store):
    """The device layout (rows per brick, incl. a ragged last brick, or the
    plain order when blocks hold several rows) changes no result: states,
    moments, wall records and statistics agree bit for bit, and a checkpoint
    taken under one layout resumes exactly under another."""
    grid = (256, 11, 5)
    h0 = _state(orc, grid, store, 11)
    one_row = (256, 256, 1) if store == "f64" else (64, 64, 4)
    segments = (128, 128, 1) if store == "f64" else (64, 64, 2)
    cfgs = [dict(tiles=one_row, brick=1), dict(tiles=one_row, brick=3), dict(tiles=one_row, brick=8),
            dict(tiles=segments, brick=8), dict(tiles=(512, 512, 1 if store == "f64" else 4), brick=8)]
    want_brick = [1, 3, 8, 8, 11]
    out = []
    for cfg, wb in zip(cfgs, want_brick):
        ch = P.Channel(*grid, 0.51, cs=0.1, fx=1e-6, store=store, bc="wfb", stats_every=2, graph_steps=0, **cfg)
        ch.set_state(h0)
        assert ch.get_param(14) == wb, cfg
        ch.step(9)
        out.append((ch.get_state(), ch.moments(), ch.wall_shear(), ch.stats_sums()[0]))
        ch.close()
    for k, o in enumerate(out[1:], 1):
        assert np.array_equal(o[0], out[0][0])
        for a, b in zip(o[1], out[0][1]):
            assert np.array_equal(a, b)
        for a, b in zip(o[2], out[0][2]):
            assert np.array_equal(a, b)
        if cfgs[k]["tiles"] == cfgs[0]["tiles"]:
            assert np.array_equal(o[3], out[0][3])
        else:   # other row segments: the same FP64 sums in another order
            np.testing.assert_allclose(o[3], out[0][3], rtol=1e-13, atol=1e-15)
    # checkpoint: bricked -> plain layout
    a = P.Channel(*grid, 0.51, cs=0.1, fx=1e-6, store=store, bc="wfb", tiles=one_row, brick=8)
    a.set_state(h0)
    a.step(5)
    saved = a.get_state()
    a.step(4)
    b = P.Channel(*grid, 0.51, cs=0.1, fx=1e-6, store=store, bc="wfb", tiles=cfgs[-1]["tiles"])
    b.set_state(saved, steps=5)
    b.step(4)
    assert np.array_equal(a.get_state(), b.get_state())


def test_layout_rejects_incompatible_blocks(P, orc):
    """Once the state is initialised in bricks, block sizes that would put
    several rows in one block are refused (and the old ones kept)."""
    ch = P.Channel(256, 11, 5, 0.51, store="f64", bc="wfb", tiles=(256, 256, 1), brick=8)
    ch.init_spalding(1e-3)
    with pytest.raises(P.LbmError) as e:
        ch.set_param(5, 512)
    assert e.value.code == -2
    assert ch.get_param(5) == 256
    ch.set_param(5, 128)          # row segments are fine
    ch.step(2)
    assert ch.sync()[0] == 0


SPREAD_CASES = [  # grid, store, tiles, odd step by rows, rows per brick: every brick whole, 32k tiles each
    ((256, 24, 32), "f16", (64, 64, 4), 0, 8),      # 3 bricks (no rotation), one row per block
    ((256, 32, 32), "bf16", (64, 64, 4), 2, 8),     # 4 bricks (rotated rounds), odd step by rows
    ((512, 32, 16), "f64", (256, 256, 1), 0, 8),    # two segments per row
    ((256, 48, 16), "f32", (128, 128, 2), 0, 4),    # 12 bricks of 4 rows
]


@pytest.mark.parametrize("grid,store,tiles,rows,brick", SPREAD_CASES)
def test_brick_spread_launch_order(P, orc, grid, store, tiles, rows, brick):
    """Spreading the bricks over the launch (chunks of 32, 128 or 256 tiles) only
    reorders the blocks: states, moments, wall records and statistics agree
    bit for bit with memory order."""
    h0 = _state(orc, grid, store, 23)
    out = []
    for spread in (0, 5, 7, 8):
        ch = P.Channel(*grid, 0.51, cs=0.1, fx=2e-6, store=store, bc="wfb", tiles=tiles, brick=brick,
                       stats_every=1, graph_steps=0)
        ch.set_param(15, rows)
        ch.set_param(16, spread)
        assert ch.get_param(16) == spread
        ch.set_state(h0)
        ch.step(7)
        assert ch.sync()[0] == 0
        out.append((ch.get_state(), ch.moments(), ch.wall_shear(), ch.stats_sums()[0]))
        ch.close()
    for o in out[1:]:
        assert np.array_equal(out[0][0], o[0])
        for a, b in zip(out[0][1], o[1]):
            assert np.array_equal(a, b)
        for a, b in zip(out[0][2], o[2]):
            assert np.array_equal(a, b)
        assert np.array_equal(out[0][3], o[3])


ROWS_CASES = [  # grid, store, tiles (odd, even, cells per thread), boundary, rows per brick
    ((256, 7, 5), "f16", (128, 128, 4), "wfb", 0),      # one 64-lane segment per row
    ((512, 6, 4), "bf16", (64, 128, 4), "wfb", 3),      # two segments, bricks of 3 rows
    ((512, 9, 3), "f32", (128, 256, 2), "freeslip", 0),  # four segments
    ((192, 5, 4), "f64", (256, 64, 1), "bb", 2),        # three segments, blocks of 4 rows
    ((128, 6, 7), "f16", (64, 64, 2), "wfb", 128),      # plain layout
]


@pytest.mark.parametrize("grid,store,tiles,bc,brick", ROWS_CASES)
def test_odd_step_by_rows_equals_blocks(P, orc, grid, store, tiles, bc, brick):
    """The odd step walking rows (one wavefront per row, edge elements carried
    across segments and around the periodic row) gives bit for bit the state,
    moments and wall records of the block kernel with its LDS exchange;
    statistics agree up to their summation order."""
    h0 = _state(orc, grid, store, 21)
    out = []
    for mode in (0, 2):
        ch = P.Channel(*grid, 0.51, cs=0.1, fx=2e-6, store=store, bc=bc, tiles=tiles, brick=brick,
                       stats_every=1, graph_steps=0)
        ch.set_param(15, mode)
        ch.set_state(h0)
        ch.step(7)
        assert ch.sync()[0] == 0
        out.append((ch.get_state(), ch.moments(), ch.wall_shear(), ch.stats_sums()[0]))
        ch.close()
    assert np.array_equal(out[0][0], out[1][0])
    for a, b in zip(out[0][1], out[1][1]):
        assert np.array_equal(a, b)
    for a, b in zip(out[0][2], out[1][2]):
        assert np.array_equal(a, b)
    np.testing.assert_allclose(out[1][3], out[0][3], rtol=1e-12, atol=1e-14)


def test_odd_step_by_rows_matches_oracle(P, orc):
    """Two FP64 steps walking rows of three segments against the oracle."""
    from gpu_common import one_step_tol, oracle_for
    w = weights(orc)
    grid = (192, 6, 3)
    h0 = _state(orc, grid, "f64", 22)
    ch = P.Channel(*grid, 0.52, cs=0.1, fx=1e-6, store="f64", bc="wfb", tiles=(128, 128, 1))
    ch.set_param(15, 2)
    ch.set_state(h0)
    ch.step(2)
    o = oracle_for(orc, grid, 0.52, 0.1, 1e-6, "wfb")
    o.set_state(h0 + w)
    assert o.step(2) == 0
    want = o.state() - w
    assert np.all(np.abs(ch.get_state() - want) <= 4 * one_step_tol("f64", want, w))


def test_batch_odd_step_by_rows(P):
    """A batch whose rows all qualify walks rows in its odd step and still
    equals each channel stepped alone."""
    specs = [dict(nx=128, ny=6, nz=3, tau=0.51, cs=0.1, fx=1e-6, bc="wfb"),
             dict(nx=256, ny=5, nz=4, tau=0.52, cs=0.1, fx=2e-6, bc="bb")]
    b = P.Batch(specs, store="f32", tiles=(64, 128, 2), graph_steps=0)
    b._set(15, 2)
    b.init_spalding([1e-2, 2e-2], 0.05, seeds=[3, 4])
    b.step(5)
    assert b.sync()[0] == 0
    for i, s in enumerate(specs):
        ch = P.Channel(s["nx"], s["ny"], s["nz"], s["tau"], cs=s["cs"], fx=s["fx"], store="f32", bc=s["bc"],
                       tiles=(64, 128, 2), graph_steps=0)
        ch.set_param(15, 0)
        ch.init_spalding([1e-2, 2e-2][i], 0.05, 3 + i)
        ch.step(5)
        assert np.array_equal(b.instance(i).get_state(), ch.get_state()), i


@pytest.mark.parametrize("graph_steps", (0, 8))
def test_empty_calls_leave_the_state_alone(P, orc, graph_steps):
    """Zero steps (single channel and batch, eager and in graphs) and an empty
    cell list are no-ops: the state, the step count and the status stay as
    they were."""
    grid = (64, 6, 3)
    h0 = _state(orc, grid, "f32", 7)
    ch = P.Channel(*grid, 0.52, cs=0.1, fx=1e-6, store="f32", bc="wfb", graph_steps=graph_steps)
    ch.set_state(h0)
    ch.step(0)
    assert ch.steps == 0 and ch.sync()[0] == 0
    np.testing.assert_array_equal(ch.get_state(), h0)
    assert ch.get_state_cells(np.zeros(0, dtype=np.int64)).shape == (0, 19)
    ch.step(3)
    h3 = ch.get_state()
    ch.step(0)
    assert ch.steps == 3
    np.testing.assert_array_equal(ch.get_state(), h3)
    b = P.Batch([dict(nx=32, ny=5, nz=3, tau=0.51, cs=0.1, fx=1e-6, bc="wfb")], store="f32", graph_steps=graph_steps)
    b.init_spalding([0.02], 0.05, seeds=[1])
    s0 = b.instance(0).get_state()
    b.step(0)
    np.testing.assert_array_equal(b.instance(0).get_state(), s0)
    assert b.sync()[0] == 0
