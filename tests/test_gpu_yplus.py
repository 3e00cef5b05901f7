"""The first-layer y+ distribution (Fig. 7) computed on the device: exact
counts against the same binning of the device's own wall records, and the
mean and standard deviation against the oracle's wall records."""
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


@pytest.mark.parametrize("store", ("f64", "f16"))
def test_yplus_pdf_counts_and_moments(P, orc, store):
    from gpu_common import oracle_for
    from paper_2009_04352_amd import workloads as W
    p = W.params("c1")
    nx, ny, nz = p["grid"]
    ch = P.Channel(nx, ny, nz, p["tau0"], cs=p["cs"], fx=p["fx"], store=store, bc="wfb")
    ch.init_spalding(p["u_tau"], p["noise"], p["seed"])
    ch.step(31)
    nbins, lo, hi = 24, -3.0, 3.0
    counts, edges, mean, std = ch.wall_yplus_pdf(nbins, lo, hi)
    assert counts.sum() == 2 * nx * nz and len(edges) == nbins + 1
    # the same binning of the device's wall records on the host
    _, _, ut, _ = ch.wall_shear()
    nu0 = (p["tau0"] - 0.5) / 3.0
    yp = (1.0 * ut.ravel()) / nu0
    assert abs(mean - yp.mean()) <= 1e-13 * mean and abs(std - yp.std()) <= 1e-11 * std
    u = ((yp - mean) / std - lo) * (nbins / (hi - lo))
    bins = np.where(~(u >= 0.0), 0, np.where(u >= nbins, nbins + 1, 1 + np.floor(np.maximum(u, 0)).astype(np.int64)))
    assert np.array_equal(counts, np.bincount(bins, minlength=nbins + 2))
    # against the oracle's wall records after the same steps (FP64 store)
    if store == "f64":
        o = oracle_for(orc, p["grid"], p["tau0"], p["cs"], p["fx"], "wfb")
        o.init_spalding(p["u_tau"], p["noise"], p["seed"])
        assert o.step(31) == 0
        _, _, uto, _ = o.wall()
        ypo = uto.ravel() / nu0
        assert abs(mean - ypo.mean()) <= 1e-11 * mean
        assert abs(std - ypo.std()) <= 1e-10 * std


def test_yplus_pdf_rejects_bad_bins(P):
    ch = P.Channel(32, 8, 4, 0.52, fx=1e-6, store="f32", bc="wfb")
    ch.init_spalding(1e-3)
    with pytest.raises(P.LbmError):
        ch.wall_yplus_pdf(0, -1.0, 1.0)
    with pytest.raises(P.LbmError):
        ch.wall_yplus_pdf(10, 1.0, 1.0)
