"""Pins of the analysis oracle (``oracle.metrics``) to things other than itself.

Distortion metrics (Sec. II, Metrics 2 and 3) and the error autocorrelation
(Sec. V) are checked against a hand-worked example, closed forms (a constant
offset, an affine map, alternating and periodic errors), library routines
for the special cases they cover (``numpy.corrcoef``, ``numpy.correlate``)
and brute force in exact rational arithmetic.  The best-layer study
(Sec. III-B, Table II) is checked against a hand-worked 2x2 example and the
closed-form hit counts of constant fields and ramps, whose n-layer prediction
errors follow from the stencil being 1 - prod_d (1 - S_d)^n (S_d the unit
shift along dimension d).
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from conftest import golden


@pytest.fixture(scope="module")
def M(oracle):
    import oracle.metrics as M
    return M


def _frac(v):
    return Fraction(int(v[0]), int(v[1]))


# ------------------------------------------------------------ quality


def test_hand_example(M):
    g = golden("hand_quality.txt")
    x = np.array([float(v) for v in g["x"][0]])
    xr = np.array([float(v) for v in g["xr"][0]])
    q = M.quality(x, xr, max_lag=3)
    assert q["rmse"] ** 2 == pytest.approx(float(_frac(g["rmse_sq_num_den"][0])), rel=1e-15)
    assert q["nrmse"] == pytest.approx(float(_frac(g["nrmse_num_den"][0])), rel=1e-15)
    assert q["psnr"] == pytest.approx(20 * math.log10(float(g["psnr_ratio"][0][0])), rel=1e-15)
    assert q["pearson"] ** 2 == pytest.approx(float(_frac(g["pearson_sq_num_den"][0])), rel=1e-14)
    assert q["pearson"] > 0
    assert q["mean_err"] == float(_frac(g["mean_err_num_den"][0]))
    assert q["max_abs_err"] == float(g["max_abs_err"][0][0])
    assert q["value_range"] == 3.0
    want = [float(_frac(v)) for v in g["autocorr_num_den"]]
    assert q["autocorr"] == pytest.approx(want, rel=1e-14)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_constant_offset(M, dtype):
    """x' = x + c: RMSE = max error = |c|, Pearson = 1, mean error = -c."""
    rng = np.random.default_rng(1)
    x = rng.integers(-1000, 1000, 5000).astype(dtype)
    c = dtype(0.375)
    q = M.quality(x, x + c)
    assert q["rmse"] == pytest.approx(0.375, rel=1e-14)
    assert q["max_abs_err"] == 0.375
    assert q["mean_err"] == pytest.approx(-0.375, rel=1e-14)
    assert q["pearson"] == pytest.approx(1.0, abs=1e-14)
    r = float(x.max()) - float(x.min())
    assert q["psnr"] == pytest.approx(20 * math.log10(r / 0.375), rel=1e-14)


def test_affine_negative_slope(M):
    """x' = a x + b with a < 0 is perfectly anti-correlated."""
    x = np.linspace(-3, 7, 1001)
    q = M.quality(x, -2.5 * x + 4.0)
    assert q["pearson"] == pytest.approx(-1.0, abs=1e-14)


def test_pearson_matches_corrcoef_and_psnr_matches_mse_form(M):
    rng = np.random.default_rng(2)
    x = rng.standard_normal(20000)
    xr = x + 0.1 * rng.standard_normal(20000)
    q = M.quality(x, xr)
    assert q["pearson"] == pytest.approx(np.corrcoef(x, xr)[0, 1], rel=1e-12)
    mse = np.mean((x - xr) ** 2)
    r = x.max() - x.min()
    assert q["psnr"] == pytest.approx(10 * np.log10(r * r / mse), rel=1e-12)
    assert q["nrmse"] == pytest.approx(np.sqrt(mse) / r, rel=1e-12)


def test_brute_force_exact_rationals(M):
    """Every sum redone in exact rational arithmetic on a tiny input."""
    rng = np.random.default_rng(3)
    x = rng.integers(-20, 20, 9).astype(np.float64) / 4
    xr = x + rng.integers(-3, 4, 9).astype(np.float64) / 8
    q = M.quality(x, xr, max_lag=4)
    X = [Fraction(v) for v in x]
    Y = [Fraction(v) for v in xr]
    n = len(X)
    E = [a - b for a, b in zip(X, Y)]
    mx, my, me = sum(X) / n, sum(Y) / n, sum(E) / n
    sxx = sum((a - mx) ** 2 for a in X)
    syy = sum((b - my) ** 2 for b in Y)
    sxy = sum((a - mx) * (b - my) for a, b in zip(X, Y))
    see = sum(e * e for e in E)
    assert q["rmse"] == pytest.approx(math.sqrt(see / n), rel=1e-15)
    assert q["pearson"] == pytest.approx(float(sxy) / math.sqrt(float(sxx * syy)), rel=1e-14)
    D = [e - me for e in E]
    s0 = sum(d * d for d in D)
    for k in range(1, 5):
        want = sum(D[i] * D[i + k] for i in range(n - k)) / s0
        assert q["autocorr"][k - 1] == pytest.approx(float(want), rel=1e-13, abs=1e-15)


def test_autocorr_alternating(M):
    """e_i = (-1)^i, N even: mean 0, lag-1 coefficient -(N-1)/N, lag 2 +(N-2)/N."""
    n = 1000
    x = np.zeros(n)
    xr = -((-1.0) ** np.arange(n))
    q = M.quality(x + np.arange(n), xr + np.arange(n), max_lag=2)
    assert q["autocorr"][0] == pytest.approx(-(n - 1) / n, rel=1e-14)
    assert q["autocorr"][1] == pytest.approx((n - 2) / n, rel=1e-14)


def test_autocorr_periodic(M):
    """e_i = cos(2 pi i / P) over whole periods: lag P gives (N - P) / N."""
    P, n = 16, 4096
    e = np.cos(2 * np.pi * np.arange(n) / P)
    x = np.arange(n, dtype=np.float64)
    q = M.quality(x, x - e, max_lag=P)
    assert q["autocorr"][P - 1] == pytest.approx((n - P) / n, rel=1e-12)
    assert q["autocorr"][P // 2 - 1] == pytest.approx(-(n - P // 2) / n, rel=1e-12)


def test_autocorr_matches_numpy_correlate_in_raster_order(M):
    """The lag runs along the raster order of a 2D array."""
    rng = np.random.default_rng(4)
    x = rng.standard_normal((37, 29))
    xr = x + 1e-3 * rng.standard_normal((37, 29))
    q = M.quality(x, xr, max_lag=40)
    d = (x - xr).ravel()
    d = d - d.mean()
    full = np.correlate(d, d, mode="full")
    want = full[d.size:d.size + 40] / full[d.size - 1]
    assert q["autocorr"] == pytest.approx(list(want), rel=1e-10, abs=1e-13)


def test_white_noise_errors_are_uncorrelated(M):
    rng = np.random.default_rng(5)
    n = 200000
    x = rng.standard_normal(n)
    q = M.quality(x, x + rng.uniform(-1e-3, 1e-3, n), max_lag=8)
    assert max(abs(v) for v in q["autocorr"]) < 5 / math.sqrt(n)


# ------------------------------------------------------------ layer survey


def test_survey_hand_example(M):
    g = golden("hand_layer_survey.txt")
    x = np.array([float(v) for v in g["x"][0]], np.float32).reshape(2, 2)
    r = M.layer_survey(x, eb_mode="abs", eb_abs=float(g["eb"][0][0]))
    want = [int(v) / 4 for v in g["rph_quarters"][0]]
    assert r["rph_orig"] == want
    assert r["rph_decomp"] == want
    assert r["best_layers"] == int(g["best"][0][0])


@pytest.mark.parametrize("shape,block", [((500,), None), ((3000,), (1000,)), ((2500,), (1000,)),
                                         ((24, 40), (12, 20)), ((25, 41), (12, 20)),
                                         ((10, 12, 14), None), ((10, 12, 14), (5, 12, 7)), ((11, 3, 14), (5, 12, 3))])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_survey_constant_field(M, shape, block, dtype):
    """A constant field of 1.0: in each independent block the n-layer error is
    nonzero exactly on the n^d points with every coordinate below n, and the
    stored misses equal 1.0, so both rates are 1 - n^d * blocks / N."""
    x = np.ones(shape, dtype)
    r = M.layer_survey(x, block=block, eb_mode="abs", eb_abs=0.01)
    N = x.size
    blk = block if block else ((2048,) if len(shape) == 1 else shape)
    for n in range(1, 5):
        # sum over blocks of prod_d min(n, block extent along d), separable per dimension
        misses = 1
        for s, b in zip(shape, blk):
            exts = [min(b, s - o) for o in range(0, s, b)]
            misses *= sum(min(n, e) for e in exts)
        want = 1 - misses / N
        assert r["rph_orig"][n - 1] == pytest.approx(want, abs=1e-15), n
        assert r["rph_decomp"][n - 1] == pytest.approx(want, abs=1e-15), n
    assert r["best_layers"] == 1


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_survey_ramp_original(M, dtype):
    """x = i along the fastest dimension (one block): with eb < 1 the n-layer
    error from original values is nonzero for i >= 1 when n = 1, and for
    1 <= i <= n - 1 (times the n^(d-1) corner of the other dimensions) when n >= 2."""
    X = 64
    x1 = np.arange(X, dtype=dtype)
    r1 = M.layer_survey(x1, eb_mode="abs", eb_abs=0.25)
    assert r1["rph_orig"] == [1 / X, (X - 1) / X, (X - 2) / X, (X - 3) / X]
    x3 = np.broadcast_to(np.arange(X, dtype=dtype), (6, 7, X)).copy()
    r3 = M.layer_survey(x3, eb_mode="abs", eb_abs=0.25)
    N = x3.size
    want = [1 - (X - 1) / N] + [1 - (n - 1) * n * n / N for n in (2, 3, 4)]
    assert r3["rph_orig"] == pytest.approx(want, abs=1e-15)


def test_survey_centred_sample_and_field_bound(M):
    """The sample is the centred sub-block; the bound is the whole field's."""
    rng = np.random.default_rng(6)
    x = rng.uniform(-50, 50, (20, 24, 30)).astype(np.float32)
    x[6:14, 8:16, 11:19] = 1.0  # the centred 8^3 sample is constant
    r = M.layer_survey(x, sample=(8, 8, 8), eb_mode="rel", eb_rel=1e-4)
    assert r["sample_shape"] == (8, 8, 8)
    want = [1 - n ** 3 / 512 for n in range(1, 5)]
    assert r["rph_orig"] == pytest.approx(want, abs=1e-15)
    assert r["rph_decomp"] == pytest.approx(want, abs=1e-15)
    rng_x = float(x.max()) - float(x.min())
    assert r["eb"] == pytest.approx(1e-4 * rng_x, rel=1e-15)
    # an absolute bound equal to the whole field's relative one gives the same study
    r2 = M.layer_survey(x, sample=(8, 8, 8), eb_mode="abs", eb_abs=r["eb"])
    assert r2["rph_decomp"] == r["rph_decomp"] and r2["rph_orig"] == r["rph_orig"]


def test_survey_decomp_rate_is_compressor_unpredictable_fraction(M, oracle):
    """rph_decomp(n) = 1 - (codes equal to 0) / N of the compressor at m = 1."""
    rng = np.random.default_rng(7)
    x = np.cumsum(rng.standard_normal((16, 40)), axis=1).astype(np.float32)
    r = M.layer_survey(x, eb_mode="abs", eb_abs=0.3)
    for n in range(1, 5):
        _, _, codes, _ = oracle.compress(x, debug=True, layers=n, m=1, eb_mode="abs", eb_abs=0.3)
        assert r["rph_decomp"][n - 1] == pytest.approx(1 - np.count_nonzero(codes == 0) / x.size, abs=1e-15)
    assert r["best_layers"] == 1 + int(np.argmax(r["rph_decomp"]))
