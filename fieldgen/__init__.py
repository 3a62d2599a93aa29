"""Seeded synthetic fields standing in for the paper's data sets.

The paper evaluates on climate (ATM, 1800x3600), X-ray (APS) and hurricane
fields (Sec. V, Table III) that are not available here.  These generators make
fields of the same shapes and kinds of structure from a seed; they hold none of
the compressor's arithmetic and are shared by the tests, the smoke check and
the benchmark.

Recipes (all generated in float64 with numpy PCG64 and cast at the end unless
noted; the Gaussian random fields are made in float32 to bound host memory):

* ``smooth3d``   - sum of 8 random 3D Gaussians (amplitude U[0.5,2], width
  U[4,16], centre U[0,n)) + sin(0.1x)cos(0.07y)sin(0.05z) on integer indices
  (x fastest) + N(0, 1e-3) noise.
* ``climate2d``  - 280 - 30 sin^2(lat) with lat at cell centres in [-90, 90],
  plus a periodic Gaussian random field with power spectrum k^-2.5 (std 5),
  plus 1% of points (chosen without replacement) offset by U[-50, 50].
* ``cosmo3d``    - lognormal density exp(g), g a Gaussian random field with
  spectrum k^-3 and std 1.5; ``velocity3d`` a separate zero-mean field with the
  same spectrum and std 300.
* ``batch_fields`` - 64 fields: 32 square 2D fields of side log-uniform in
  [512, 4096] (climate recipe) and 32 cubes of side log-uniform in [64, 384]
  (smooth recipe), each with a log-uniform relative bound in [1e-5, 1e-3].
* ``request_stream`` - Poisson arrivals of compress/decompress requests with
  lognormal sizes (median 32 MB, sigma 1.5, clipped to [1 MB, 2 GB]).
"""
from __future__ import annotations

import math

import numpy as np

BASE_SEED = 20170612


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def smooth3d(shape=(64, 64, 64), seed=BASE_SEED + 0, dtype=np.float32) -> np.ndarray:
    g = rng(seed)
    nz, ny, nx = shape
    z = np.arange(nz, dtype=np.float64)[:, None, None]
    y = np.arange(ny, dtype=np.float64)[None, :, None]
    x = np.arange(nx, dtype=np.float64)[None, None, :]
    out = np.zeros(shape, np.float64)
    for _ in range(8):
        a = g.uniform(0.5, 2.0)
        w = g.uniform(4.0, 16.0)
        cz, cy, cx = g.uniform(0, nz), g.uniform(0, ny), g.uniform(0, nx)
        out += a * np.exp(-((z - cz) ** 2 + (y - cy) ** 2 + (x - cx) ** 2) / (2 * w * w))
    out += np.sin(0.1 * x) * np.cos(0.07 * y) * np.sin(0.05 * z)
    out += g.normal(0.0, 1e-3, size=shape)
    return out.astype(dtype)


def _grf(shape, slope, std, g: np.random.Generator) -> np.ndarray:
    """Periodic Gaussian random field with power spectrum |k|^slope, P(0) = 0."""
    import scipy.fft as sfft

    white = g.standard_normal(shape, dtype=np.float32)
    spec = sfft.rfftn(white, workers=-1)
    del white
    k2 = None
    for ax, n in enumerate(shape):
        if ax == len(shape) - 1:
            f = np.fft.rfftfreq(n).astype(np.float32)
        else:
            f = np.fft.fftfreq(n).astype(np.float32)
        sh = [1] * len(shape)
        sh[ax] = len(f)
        term = (f * f).reshape(sh)
        k2 = term if k2 is None else k2 + term
    # amplitude ~ k^(slope/2); computed in place over the broadcast grid
    amp = np.empty(spec.shape, np.float32)
    amp[...] = k2
    amp.flat[0] = 1.0
    np.power(amp, np.float32(slope / 4.0), out=amp)
    amp.flat[0] = 0.0
    spec *= amp
    del amp
    field = sfft.irfftn(spec, s=shape, workers=-1).astype(np.float32, copy=False)
    del spec
    field -= np.float32(field.mean(dtype=np.float64))
    sd = float(field.std(dtype=np.float64))
    field *= np.float32(std / sd)
    return field


def climate2d(shape=(1800, 3600), seed=BASE_SEED + 1, dtype=np.float32) -> np.ndarray:
    g = rng(seed)
    ny, nx = shape
    lat = np.deg2rad(-90.0 + (np.arange(ny) + 0.5) * 180.0 / ny)[:, None]
    base = 280.0 - 30.0 * np.sin(lat) ** 2
    out = base + _grf(shape, -2.5, 5.0, g).astype(np.float64)
    n = ny * nx
    nsp = max(1, n // 100)
    idx = g.choice(n, size=nsp, replace=False)
    out.reshape(-1)[idx] += g.uniform(-50.0, 50.0, size=nsp)
    return out.astype(dtype)


def cosmo3d(shape=(512, 512, 512), seed=BASE_SEED + 2, dtype=np.float32) -> np.ndarray:
    g = rng(seed)
    f = _grf(shape, -3.0, 1.5, g)
    np.exp(f, out=f)
    return f.astype(dtype, copy=False)


def velocity3d(shape=(512, 512, 512), seed=BASE_SEED + 102, dtype=np.float32) -> np.ndarray:
    g = rng(seed)
    return _grf(shape, -3.0, 300.0, g).astype(dtype, copy=False)


def batch_fields(count=64, seed=BASE_SEED + 3, scale=1.0):
    """Specs of the uneven batch: list of dicts (shape, eb_rel, seed, kind).

    ``scale`` shrinks the sides (for quick tests); 1.0 is the full mix.
    """
    g = rng(seed)
    specs = []
    for i in range(count):
        if i % 2 == 0:
            side = int(round(math.exp(g.uniform(math.log(512), math.log(4096))) * scale))
            shape = (max(side, 8), max(side, 8))
            kind = "climate2d"
        else:
            side = int(round(math.exp(g.uniform(math.log(64), math.log(384))) * scale))
            shape = (max(side, 4),) * 3
            kind = "smooth3d"
        eb = math.exp(g.uniform(math.log(1e-5), math.log(1e-3)))
        specs.append({"shape": shape, "eb_rel": eb, "seed": seed * 1000 + i, "kind": kind})
    return specs


def make_batch_field(spec, dtype=np.float32) -> np.ndarray:
    if spec["kind"] == "climate2d":
        return climate2d(spec["shape"], spec["seed"], dtype)
    return smooth3d(spec["shape"], spec["seed"], dtype)


def near_cubic(n_points: int, ndim: int):
    """A shape of about n_points elements with near-equal sides."""
    if ndim == 1:
        return (n_points,)
    side = max(2, int(round(n_points ** (1.0 / ndim))))
    if ndim == 2:
        return (max(1, n_points // side), side)
    return (max(1, n_points // (side * side)), side, side)


def request_stream(rate: float, duration: float, seed=BASE_SEED + 4, size_scale=1.0,
                   max_bytes=2 << 30, min_bytes=1 << 20):
    """Poisson arrivals: list of dicts (t_arrival, op, dtype, shape, eb_rel, seed)."""
    g = rng(seed)
    t = 0.0
    out = []
    i = 0
    while True:
        t += g.exponential(1.0 / rate)
        if t > duration:
            break
        nbytes = math.exp(g.normal(math.log(32e6), 1.5)) * size_scale
        nbytes = min(max(nbytes, min_bytes * size_scale), max_bytes * size_scale)
        dt = np.float32 if g.uniform() < 0.8 else np.float64
        ndim = int(g.integers(1, 4))
        npts = max(64, int(nbytes // np.dtype(dt).itemsize))
        shape = near_cubic(npts, ndim)
        eb = math.exp(g.uniform(math.log(1e-6), math.log(1e-3)))
        op = "compress" if g.uniform() < 0.5 else "decompress"
        out.append({"t": t, "op": op, "dtype": dt, "shape": shape, "eb_rel": eb,
                    "seed": seed * 100000 + i})
        i += 1
    return out


def request_field(req) -> np.ndarray:
    """Field data of a request: smooth recipe for 3D, climate-like for 2D, 1D cut."""
    shape, dt, sd = req["shape"], req["dtype"], req["seed"]
    g = rng(sd)
    if len(shape) == 1:
        n = shape[0]
        xs = np.arange(n, dtype=np.float64)
        base = np.sin(xs * 0.001) * 10 + np.cumsum(g.normal(0, 0.05, n))
        return base.astype(dt)
    if len(shape) == 2:
        ny, nx = shape
        yy = np.arange(ny, dtype=np.float64)[:, None]
        xx = np.arange(nx, dtype=np.float64)[None, :]
        f = 280 + 10 * np.sin(yy * 0.01) * np.cos(xx * 0.013) + g.normal(0, 0.05, shape)
        return f.astype(dt)
    nz, ny, nx = shape
    zz = np.arange(nz, dtype=np.float64)[:, None, None]
    yy = np.arange(ny, dtype=np.float64)[None, :, None]
    xx = np.arange(nx, dtype=np.float64)[None, None, :]
    f = np.sin(0.05 * xx) * np.cos(0.04 * yy) * np.sin(0.03 * zz) + g.normal(0, 1e-3, shape)
    return f.astype(dt)
