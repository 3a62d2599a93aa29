"""Parity of the analysis entry points with the oracle (MI355X only).

``sz_quality`` (Sec. II Metrics 2-3, Sec. V error autocorrelation) sums in a
different order than the oracle (numpy's pairwise sums), so its double results
may differ by rounding.  The device adds at most about 256 terms per thread,
then 6 + 2 tree levels, then at most 2048 block partials (40 000 terms per
block partial plus block count for the autocorrelation at 512^3), so each sum
is within about 4e4 * 2^-53 < 1e-11 of exact relative to the sum of the
magnitudes of its terms, and numpy is closer still.  With that: RMSE, NRMSE
and PSNR (sums of squares) are checked relatively; Pearson's coefficient and
the autocorrelation, whose mixed-sign numerators are bounded by their
denominators (Cauchy-Schwarz), absolutely; the mean error absolutely against
the maximum error.  1e-9 leaves a margin of 100 over the bound.  Minimum,
maximum and maximum error are exact.  ``sz_layer_survey`` (Sec. III-B,
Table II) counts points, so its rates equal the oracle's exactly.
"""
import numpy as np
import pytest

import fieldgen as F

pytestmark = pytest.mark.gpu

REL = 1e-9


@pytest.fixture(scope="module")
def Z():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    import paper_1706_03791_amd as Z
    Z.lib()
    return Z


@pytest.fixture(scope="module")
def M(oracle):
    import oracle.metrics as M
    return M


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def recon(Z, x, **kw):
    comp, _ = Z.compress(dev(x), **kw)
    return Z.decompress(comp).cpu().numpy().reshape(x.shape)


def check_quality(Z, M, x, xr, lag):
    g = Z.quality(dev(x), dev(xr), max_lag=lag)
    r = M.quality(x, xr, max_lag=lag)
    for k in ("value_min", "value_max", "value_range", "max_abs_err"):
        assert g[k] == r[k], (k, g[k], r[k])
    assert g["n"] == r["n"]
    for k in ("rmse", "nrmse", "psnr"):
        assert g[k] == pytest.approx(r[k], rel=REL), k
    assert g["pearson"] == pytest.approx(r["pearson"], abs=REL)
    scale = r["max_abs_err"]
    assert g["mean_err"] == pytest.approx(r["mean_err"], rel=REL, abs=REL * scale)
    if lag:
        assert g["autocorr"] == pytest.approx(r["autocorr"], abs=REL)
    return g


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("shape", [(64, 64, 64), (19, 37, 45), (90, 130), (10007,), (4096,), (4097,)])
def test_quality_of_reconstruction(Z, M, shape, dtype):
    x = F.smooth3d(shape if len(shape) == 3 else (1, 1, int(np.prod(shape))), seed=F.BASE_SEED + 11,
                   dtype=dtype).reshape(shape)
    xr = recon(Z, x, eb_mode="rel", eb_rel=1e-3)
    q = check_quality(Z, M, x, xr, lag=32)
    assert q["max_abs_err"] <= 1e-3 * q["value_range"]


@pytest.mark.parametrize("n", [2, 3, 255, 256, 257, 4095 + 255])
def test_quality_small_and_ragged(Z, M, n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n)
    xr = x + 1e-2 * rng.standard_normal(n)
    check_quality(Z, M, x, xr, lag=min(255, n - 1))


def test_quality_closed_forms(Z):
    x = np.arange(4096, dtype=np.float32)
    q = Z.quality(dev(x), dev(x + np.float32(0.375)), max_lag=0)
    assert q["rmse"] == 0.375 and q["max_abs_err"] == 0.375
    assert q["pearson"] == pytest.approx(1.0, abs=1e-14)
    xr = x + np.where(np.arange(4096) % 2 == 0, 1, -1).astype(np.float32)
    q = Z.quality(dev(x), dev(xr), max_lag=2)
    assert q["autocorr"][0] == pytest.approx(-4095 / 4096, rel=1e-14)
    assert q["autocorr"][1] == pytest.approx(4094 / 4096, rel=1e-14)


def test_quality_rejects_bad_arguments(Z):
    x = dev(np.zeros(8, np.float32))
    ctx = Z.context(0)
    rc, _, _ = Z.sz_quality(ctx, Z.SZ_F32, 1, x.data_ptr(), x.data_ptr(), 0)
    assert rc == Z.SZ_EINVAL
    rc, _, _ = Z.sz_quality(ctx, Z.SZ_F32, 8, x.data_ptr(), x.data_ptr(), 256)
    assert rc == Z.SZ_EINVAL
    rc, _, _ = Z.sz_quality(ctx, 7, 8, x.data_ptr(), x.data_ptr(), 0)
    assert rc == Z.SZ_EINVAL


def test_quality_full_size_cosmology(Z, M):
    """The 512^3 single-precision field at a relative bound of 1e-4."""
    import fieldgen.gpu as G
    import torch
    x = G.cosmo3d((512, 512, 512), F.BASE_SEED + 2)
    comp, _ = Z.compress(x, eb_mode="rel", eb_rel=1e-4)
    xr = Z.decompress(comp).view(x.shape)
    g = Z.quality(x, xr, max_lag=2)
    torch.cuda.synchronize()
    r = M.quality(x.cpu().numpy(), xr.cpu().numpy(), max_lag=2)
    for k in ("value_min", "value_max", "max_abs_err"):
        assert g[k] == r[k], k
    for k in ("rmse", "psnr"):
        assert g[k] == pytest.approx(r[k], rel=REL), k
    assert g["pearson"] == pytest.approx(r["pearson"], abs=REL)
    assert g["autocorr"] == pytest.approx(r["autocorr"], abs=REL)
    assert g["max_abs_err"] <= 1e-4 * g["value_range"]


def check_survey(Z, M, x, sample=None, **kw):
    g = Z.layer_survey(dev(x), sample=sample, **kw)
    r = M.layer_survey(x, sample=sample, **kw)
    assert g["rph_decomp"] == r["rph_decomp"]
    assert g["rph_orig"] == r["rph_orig"]
    assert g["best_layers"] == r["best_layers"]
    return g


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("shape,sample,block", [
    ((64, 64, 64), None, None), ((64, 64, 64), (32, 32, 32), None), ((33, 70, 129), (20, 31, 64), (8, 16, 32)),
    ((90, 130), None, None), ((300, 257), (101, 99), (50, 64)), ((10007,), None, None), ((10007,), (3001,), (1000,)),
])
def test_survey_parity(Z, M, shape, sample, block, dtype):
    x = F.smooth3d(shape if len(shape) == 3 else (1, 1, int(np.prod(shape))), seed=F.BASE_SEED + 12,
                   dtype=dtype).reshape(shape)
    check_survey(Z, M, x, sample=sample, block=block, eb_mode="rel", eb_rel=1e-4)


def test_survey_constant_closed_form(Z):
    x = np.ones((10, 12, 14), np.float32)
    g = Z.layer_survey(dev(x), eb_mode="abs", eb_abs=0.01)
    want = [1 - n ** 3 / x.size for n in range(1, 5)]
    assert g["rph_decomp"] == pytest.approx(want, abs=1e-15)
    assert g["rph_orig"] == pytest.approx(want, abs=1e-15)
    assert g["best_layers"] == 1


def test_survey_full_size_cosmology_sample(Z, M):
    """A centred 64^3 sample of the 512^3 field, the bound taken on the whole field."""
    import fieldgen.gpu as G
    x = G.cosmo3d((512, 512, 512), F.BASE_SEED + 2)
    g = Z.layer_survey(x, sample=(64, 64, 64), eb_mode="rel", eb_rel=1e-4)
    r = M.layer_survey(x.cpu().numpy(), sample=(64, 64, 64), eb_mode="rel", eb_rel=1e-4)
    assert g["rph_decomp"] == r["rph_decomp"]
    assert g["rph_orig"] == r["rph_orig"]
    assert g["best_layers"] == r["best_layers"]


def test_rate_distortion_invariants(Z):
    """Over decreasing relative bounds on the climate-like field: the maximum
    error stays within the bound (Metric 1), so PSNR > 20 log10(1 / eb_rel);
    PSNR rises and the bit-rate does not fall."""
    import math
    import fieldgen.gpu as G
    x = G.climate2d((360, 720), F.BASE_SEED + 1)
    prev = None
    for eb in (1e-2, 1e-3, 1e-4, 1e-5, 1e-6):
        comp, st = Z.compress(x, layers=1, m=0, eb_mode="rel", eb_rel=eb)
        xr = Z.decompress(comp).view(x.shape)
        q = Z.quality(x, xr)
        assert q["max_abs_err"] <= st["eb_used"]
        assert q["psnr"] > 20 * math.log10(1 / eb)
        bits = 8.0 * comp.numel() / x.numel()
        if prev:
            assert q["psnr"] > prev[0] and bits >= prev[1], (eb, q["psnr"], bits, prev)
        prev = (q["psnr"], bits)


def test_survey_smooth_field_prefers_more_layers_on_original_values(Z, M):
    """On the smooth separable-sine field, original neighbours favour two or
    more layers while decompressed neighbours favour one (Table II's effect)."""
    import fieldgen.gpu as G
    x = G.sines3d((64, 64, 64))
    g = Z.layer_survey(x, eb_mode="rel", eb_rel=1e-4)
    r = M.layer_survey(x.cpu().numpy(), eb_mode="rel", eb_rel=1e-4)
    assert g["rph_decomp"] == r["rph_decomp"] and g["rph_orig"] == r["rph_orig"]
    assert g["best_layers"] == 1
    assert max(range(4), key=lambda n: g["rph_orig"][n]) >= 1
