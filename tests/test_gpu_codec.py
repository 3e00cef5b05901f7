"""The store formats' device codec (the conversion code of the step kernels)
rounds to nearest with ties to even, keeps subnormals, and is exact for FP32."""
import numpy as np
import pytest

from gpu_common import round_to

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_04352_amd as P
    return P


def _ties(store, rng, n):
    """float32 values exactly halfway between two neighbours of the store format."""
    if store == "bf16":
        hi = rng.integers(0x0080, 0x7f00, n).astype(np.uint32) << 16
        return (hi | 0x8000).view(np.float32)
    base = rng.uniform(6.2e-5, 6e4, n).astype(np.float16).astype(np.float32)
    nxt = np.nextafter(base.astype(np.float16), np.float16(np.inf)).astype(np.float32)
    return ((base.astype(np.float64) + nxt) / 2).astype(np.float32)


@pytest.mark.parametrize("store", ("f32", "f16", "bf16"))
def test_codec_rounds_to_nearest_even(P, store):
    rng = np.random.default_rng(31)
    vals = np.concatenate([
        rng.normal(0, 1e-2, 4000), rng.normal(0, 1e-5, 2000), rng.normal(0, 1.0, 1000),
        [0.0, -0.0, 1.0, -1.0, 2.0 ** -24, 3 * 2.0 ** -25, 6.1e-5, 65504.0, 1e-3, -1e-3],
    ]).astype(np.float32)
    if store != "f32":
        vals = np.concatenate([vals, _ties(store, rng, 3000), -_ties(store, rng, 1000)])
    got = P.codec_roundtrip(store, vals)
    want = round_to(store, vals.astype(np.float64)).astype(np.float32)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def test_codec_nan_and_inf(P):
    vals = np.array([np.inf, -np.inf, np.nan], dtype=np.float32)
    for store in ("f32", "f16", "bf16"):
        got = P.codec_roundtrip(store, vals)
        assert got[0] == np.inf and got[1] == -np.inf and np.isnan(got[2])
    got = P.codec_roundtrip("f16", np.array([7e4, -7e4], dtype=np.float32))
    assert np.all(np.isinf(got))   # beyond the binary16 range


@pytest.mark.parametrize("nbytes", (16, 16 * 1023, 16 * 1024 * 33 + 48, (1 << 26) + 16 * 7))
def test_copy_probe_copies_and_runs_in_place(P, nbytes):
    """The bandwidth probe copies exactly nbytes (ragged last chunk included)
    between two buffers, leaves the bytes after them alone, and an in-place
    pass (dst == src) leaves the data unchanged."""
    import torch
    print("copy probe %d bytes" % nbytes, flush=True)
    g = torch.Generator(device="cpu").manual_seed(nbytes)
    src = torch.randint(0, 256, (nbytes + 64,), dtype=torch.uint8, generator=g).cuda()
    dst = torch.zeros(nbytes + 64, dtype=torch.uint8, device="cuda")
    P.copy_probe(dst, src, nbytes)
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes], src[:nbytes])
    assert int(dst[nbytes:].abs().sum()) == 0
    ref = src.clone()
    P.copy_probe(src, src, nbytes)
    torch.cuda.synchronize()
    assert torch.equal(src, ref)
