"""Batched ensembles: every instance of a batched launch evolves exactly (bit
for bit) as the same channel stepped alone with the same launch shape, and
matches the oracle; failures are attributed to their instance."""
import numpy as np
import pytest

from gpu_common import one_step_tol, oracle_for, random_state, weights

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_04352_amd as P
    return P


SPECS = [
    dict(nx=32, ny=9, nz=3, tau=0.51, cs=0.1, fx=1e-6, bc="wfb"),
    dict(nx=64, ny=16, nz=4, tau=0.52, cs=0.1, fx=2e-6, bc="bb"),
    dict(nx=128, ny=5, nz=2, tau=0.53, cs=0.0, fx=0.0, bc="freeslip"),
    dict(nx=96, ny=6, nz=5, tau=0.505, cs=0.2, fx=3e-6, bc="wfb"),
    dict(nx=200, ny=4, nz=3, tau=0.6, cs=0.1, fx=-1e-6, bc="bb"),
    dict(nx=16, ny=3, nz=7, tau=0.51, cs=0.1, fx=1e-6, bc="wfb"),
]


@pytest.mark.parametrize("store,tiles", [("f32", (64, 128, 2)), ("f16", (128, 64, 4)), ("f64", (256, 64, 1)),
                                         ("bf16", (64, 64, 2))])
def test_batch_equals_single(P, store, tiles):
    u_tau = [1e-2, 2e-2, 0.0, 5e-3, 1e-2, 3e-2]
    b = P.Batch(SPECS, store=store, tiles=tiles, graph_steps=4)
    b.init_spalding(u_tau, 0.05, seeds=list(range(10, 16)))
    b.step(3)
    b.step(8)     # graph chunks from both parities
    assert b.sync()[0] == 0
    for i, s in enumerate(SPECS):
        ch = P.Channel(s["nx"], s["ny"], s["nz"], s["tau"], cs=s["cs"], fx=s["fx"], store=store, bc=s["bc"],
                       tiles=tiles, graph_steps=0)
        ch.init_spalding(u_tau[i], 0.05, 10 + i)
        ch.step(11)
        v = b.instance(i)
        assert np.array_equal(v.get_state(), ch.get_state()), i
        for a, c in zip(v.moments(), ch.moments()):
            assert np.array_equal(a, c)
        assert v.steps == 11


def test_batch_matches_oracle(P, orc):
    w = weights(orc)
    specs = SPECS[:4]
    b = P.Batch(specs, store="f64", tiles=(64, 64, 1))
    b.init_spalding([1e-2, 2e-2, 0.0, 5e-3], 0.05, seeds=[1, 2, 3, 4])
    b.step(2)
    for i, s in enumerate(specs):
        o = oracle_for(orc, (s["nx"], s["ny"], s["nz"]), s["tau"], s["cs"], s["fx"], s["bc"])
        o.init_spalding([1e-2, 2e-2, 0.0, 5e-3][i], 0.05, i + 1)
        assert o.step(2) == 0
        got, want = b.instance(i).get_state(), o.state() - w
        assert np.all(np.abs(got - want) <= 4 * one_step_tol("f64", want, w)), i


def test_batch_instances_are_observation_only(P):
    b = P.Batch(SPECS[:2], store="f32")
    b.init_spalding([1e-2, 1e-2], 0.05)
    v = b.instance(1)
    with pytest.raises(P.LbmError):
        v.step(1)
    with pytest.raises(P.LbmError):
        v.set_boundary("wfb")
    with pytest.raises(P.LbmError):
        v.init_spalding(1e-3)


def test_batch_failure_names_its_instance(P, orc):
    specs = [dict(s) for s in SPECS[:3]]
    specs[2]["fx"] = 1e30          # drives instance 2 non-finite at once
    b = P.Batch(specs, store="f32", graph_steps=0)
    b.init_spalding([1e-2, 1e-2, 1e-2], 0.05)
    b.step(3)
    st, first, inst = b.sync()
    # step 1's collision overflows; the density that each step computes from its
    # gathered populations is first non-finite in step 2
    assert st == -5 and inst == 2 and first == 2


def test_ensemble_workload_runs(P):
    """The 64-channel ensemble, batched, against three of its channels run alone."""
    from paper_2009_04352_amd import workloads as W
    ens = W.ensemble()
    tiles = (256, 256, 2)
    b = P.Batch(ens, store="f32", tiles=tiles, graph_steps=8)
    b.init_spalding([e["u_tau"] for e in ens], 0.05, seeds=[e["seed"] for e in ens])
    b.step(20)
    assert b.sync()[0] == 0
    for i in (0, 17, 63):
        e = ens[i]
        ch = P.Channel(e["nx"], e["ny"], e["nz"], e["tau"], cs=e["cs"], fx=e["fx"], store="f32", bc=e["bc"],
                       tiles=tiles)
        ch.init_spalding(e["u_tau"], 0.05, e["seed"])
        ch.step(20)
        assert np.array_equal(b.instance(i).get_state(), ch.get_state()), i


def test_batch_autotune_picks_valid_shapes(P):
    """The batch tuner's choice is a valid launch shape (block sizes, cells per
    thread, odd-step mode) and the tuned batch evolves bit for bit as the
    batch with its default shapes."""
    specs = [dict(nx=128, ny=6, nz=3, tau=0.51, cs=0.1, fx=1e-6, bc="wfb"),
             dict(nx=256, ny=5, nz=4, tau=0.52, cs=0.1, fx=2e-6, bc="bb")]
    u_tau = [1e-2, 2e-2]
    tuned = P.Batch(specs, store="f32", graph_steps=0)
    t = tuned.autotune(steps=4)
    assert t[0] in (64, 128, 256, 512) and t[1] in (64, 128, 256, 512) and t[2] in (1, 2)
    out = []
    for b in (tuned, P.Batch(specs, store="f32", graph_steps=0)):
        b.init_spalding(u_tau, 0.05, seeds=[3, 4])
        b.step(5)
        assert b.sync()[0] == 0
        out.append([b.instance(i).get_state() for i in range(len(specs))])
    for a, c in zip(*out):
        np.testing.assert_array_equal(a, c)


def test_ensemble_in_its_benchmark_shapes_matches_oracle(P, orc):
    """The 64-channel ensemble in the launch shapes the benchmark's tuner picks
    for it: an odd and an even step of four instances (WFB and bounce-back
    channels of different sizes) against the oracle continued from the GPU's
    state, to the one-step tolerance."""
    from paper_2009_04352_amd import workloads as W
    ens = W.ensemble()
    b = P.Batch(ens, store="f32", graph_steps=0)
    tiles = b.autotune(steps=6)
    print("ensemble in tuned shapes", tiles, flush=True)
    b.init_spalding([e["u_tau"] for e in ens], 0.05, seeds=[e["seed"] for e in ens])
    b.step(1)
    w = weights(orc)
    sel = (0, 17, 42, 63)
    for _ in range(2):
        prev = {i: b.instance(i).get_state() for i in sel}
        b.step(1)
        for i in sel:
            e = ens[i]
            o = oracle_for(orc, (e["nx"], e["ny"], e["nz"]), e["tau"], e["cs"], e["fx"], e["bc"])
            o.set_state(prev[i] + w)
            assert o.step(1) == 0
            want = o.state() - w
            got = b.instance(i).get_state()
            assert np.all(np.abs(got - want) <= one_step_tol("f32", want, w)), (i, np.abs(got - want).max())
    assert b.sync()[0] == 0
    b.close()
