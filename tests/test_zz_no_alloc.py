"""The allocation-free y+ distribution (lbm_wall_yplus_pdf_noalloc: the
library's fixed per-device work area instead of device allocations) against
lbm_wall_yplus_pdf on the same state: the same counts and the same mean and
standard deviation, bit for bit, since both run the same kernels in the same
order.  Two calls in a row, the second on a smaller channel with fewer bins,
into output tensors filled with garbage first (the kernels clear the
counters; the work area keeps the previous call's values beyond the smaller
grid's wall cells, which must not leak in); then the first channel again."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_04352_amd as P
    return P


def _channel(P, nx, ny, nz, store, bc, steps, seed):
    from paper_2009_04352_amd import workloads as W
    p = W.params("c1")
    ch = P.Channel(nx, ny, nz, p["tau0"], cs=p["cs"], fx=p["fx"], store=store, bc=bc)
    ch.init_spalding(p["u_tau"], p["noise"], seed)
    ch.step(steps)
    assert ch.sync()[0] == 0
    return ch


def _compare(ch, nbins, lo, hi):
    import torch
    want_counts, _, want_mean, want_std = ch.wall_yplus_pdf(nbins, lo, hi)
    counts = torch.full((nbins + 2,), -7, dtype=torch.int64, device=ch.device)
    ms = torch.full((2,), float("nan"), dtype=torch.float64, device=ch.device)
    ch.wall_yplus_pdf_noalloc(counts, ms, nbins, lo, hi)
    ch.stream.synchronize()
    got = counts.cpu().numpy()
    np.testing.assert_array_equal(got, want_counts)
    assert got.sum() == 2 * ch.nx * ch.nz
    got_ms = ms.cpu().numpy()
    assert got_ms[0] == want_mean and got_ms[1] == want_std, (got_ms, want_mean, want_std)
    assert np.isfinite(want_mean) and want_std > 0


def test_noalloc_matches_allocating_entry_twice(P):
    print("no-alloc y+ pdf: 96x20x64 f32 wfb, then 40x12x24 f64 bb", flush=True)
    big = _channel(P, 96, 20, 64, "f32", "wfb", 12, 11)
    _compare(big, 40, -4.0, 4.0)
    small = _channel(P, 40, 12, 24, "f64", "bb", 7, 12)
    _compare(small, 9, -3.0, 3.0)
    _compare(big, 40, -4.0, 4.0)
    big.close()
    small.close()


def test_noalloc_rejects_host_outputs(P):
    print("no-alloc y+ pdf: host outputs rejected", flush=True)
    import torch
    from paper_2009_04352_amd import _lib as L
    ch = _channel(P, 16, 8, 8, "f64", "wfb", 2, 3)
    counts = torch.zeros(10, dtype=torch.int64)
    ms = torch.zeros(2, dtype=torch.float64)
    with pytest.raises(L.LbmError):
        ch.wall_yplus_pdf_noalloc(counts, ms, 8)
    # the rejected pointer query leaves no error behind for the next launch
    _compare(ch, 8, -4.0, 4.0)
    ch.close()
