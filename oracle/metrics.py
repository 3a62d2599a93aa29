"""TEST INFRASTRUCTURE ONLY: plain numpy (fp64) oracle of the analysis metrics.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module.  It shares no code with the HIP library.

* ``quality``: the distortion metrics of Sec. II (Metric 2: RMSE, NRMSE with
  the value range R_X, PSNR = 20 log10(R_X / RMSE); Metric 3: the Pearson
  correlation coefficient between the original and the reconstruction) and the
  autocorrelation of the compression errors that Sec. V studies, each written
  out from its textbook definition in double precision.
* ``layer_survey``: the best-layer study of Sec. III-B (Table II): the
  prediction hitting rate of n = 1..4 layers when predicting from decompressed
  values (what the compressor sees) and from original values, with a single
  interval around the prediction (the quantizer of Sec. IV-A at m = 1).
"""
from __future__ import annotations

import numpy as np

from . import predict_original, quantize, resolve_eb


def quality(x: np.ndarray, xr: np.ndarray, max_lag: int = 0) -> dict:
    """Metrics of a reconstruction ``xr`` of ``x`` (same shape), in float64.

    e_i = x_i - xr_i; R_X = max(x) - min(x);
    rmse = sqrt(sum e_i^2 / N); nrmse = rmse / R_X; psnr = 20 log10(R_X / rmse);
    pearson = sum (x_i - mean x)(xr_i - mean xr) / sqrt(sum (x_i - mean x)^2 sum (xr_i - mean xr)^2);
    autocorr[k-1] = sum_{i < N-k} d_i d_{i+k} / sum_i d_i^2, d = e - mean(e), k = 1..max_lag,
    with i running over the raster (row-major) order.
    """
    a = np.asarray(x, dtype=np.float64).ravel()
    b = np.asarray(xr, dtype=np.float64).ravel()
    if a.shape != b.shape or a.size < 2:
        raise ValueError("x and xr need the same size >= 2")
    n = a.size
    e = a - b
    vmin, vmax = a.min(), a.max()
    rng = vmax - vmin
    rmse = np.sqrt(np.sum(e * e) / n)
    da = a - np.sum(a) / n
    db = b - np.sum(b) / n
    pearson = np.sum(da * db) / np.sqrt(np.sum(da * da) * np.sum(db * db))
    with np.errstate(divide="ignore", invalid="ignore"):
        out = {
            "n": n,
            "value_min": float(vmin),
            "value_max": float(vmax),
            "value_range": float(rng),
            "max_abs_err": float(np.max(np.abs(e))),
            "mean_err": float(np.sum(e) / n),
            "rmse": float(rmse),
            "nrmse": float(rmse / rng),
            "psnr": float(20.0 * np.log10(rng / rmse)),
            "pearson": float(pearson),
        }
        if max_lag:
            d = e - np.sum(e) / n
            s0 = np.sum(d * d)
            out["autocorr"] = [float(np.sum(d[: n - k] * d[k:]) / s0) for k in range(1, max_lag + 1)]
    return out


def _sample(x: np.ndarray, sample):
    """The centred sub-block of extents ``sample`` (0 or None = whole extent)."""
    sl = []
    for d, full in enumerate(x.shape):
        s = full
        if sample is not None and d < len(sample) and sample[d] and sample[d] < full:
            s = int(sample[d])
        o = (full - s) // 2
        sl.append(slice(o, o + s))
    return np.ascontiguousarray(x[tuple(sl)])


def _sample_block(shape, sshape, block):
    """Independent blocks of the sample: the field's blocks clipped to the sample."""
    out = []
    for d, s in enumerate(sshape):
        if block is not None and block[d]:
            b = int(block[d])
        else:
            b = 2048 if len(shape) == 1 else shape[d]
        out.append(min(b, s))
    return out


def layer_survey(x: np.ndarray, sample=None, block=None, **eb) -> dict:
    """R_PH of n = 1..4 layers on the centred sample of ``x`` (Sec. III-B, Table II).

    The error bound is that of the whole field (``eb`` as for ``resolve_eb``:
    eb_mode, eb_abs, eb_rel).  A point is a hit when the m = 1 quantizer
    accepts it: t = (x - p) * (1 / 2eb) in the element type, |t| < 1,
    round-half-even(t) = 0 and |x - p| < eb.  ``rph_decomp`` predicts from the
    values the decompressor will hold (one traversal of the compressor at
    m = 1; the unpredictable count is read off the codes); ``rph_orig``
    predicts from the original values.  ``best_layers`` is the n with the
    highest ``rph_decomp``, the smallest on ties.
    """
    x = np.ascontiguousarray(x)
    T = x.dtype.type
    E = resolve_eb(x, **eb)
    s = _sample(x, sample)
    blk = _sample_block(x.shape, s.shape, block)
    Es = resolve_eb(s, eb_mode="abs", eb_abs=E["eb"])
    ebT, inv2eb = T(Es["ebT"]), T(Es["inv2eb"])
    dec, org = [], []
    for nl in range(1, 5):
        _, _, n_unpred = quantize(s, m=1, layers=nl, eb_mode="abs", eb_abs=E["eb"], block=blk)
        dec.append(1.0 - n_unpred / s.size)
        p = predict_original(s, layers=nl, block=blk)
        t = (s - p) * inv2eb
        hit = (np.abs(t) < T(1)) & (np.rint(t) == 0) & (np.abs(s - p) < ebT)
        org.append(int(np.count_nonzero(hit)) / s.size)
    best = 1 + int(np.argmax(dec))
    return {"rph_decomp": dec, "rph_orig": org, "best_layers": best, "eb": E["eb"], "sample_shape": s.shape}
