"""Device-side versions of the synthetic field recipes (torch on the GPU).

Same recipes as the numpy generators in ``fieldgen`` (see its docstring),
drawn from a seeded ``torch.Generator`` on the device instead of numpy PCG64
(Gaussian random fields on the next power-of-two grid, cropped),
so that the large inputs of the batched and served benchmarks (gigabytes of
fields) are made in milliseconds.  The values differ from the numpy
generators' for the same seed; both are deterministic.  Nothing here is part
of the compressor.
"""
from __future__ import annotations

import math


def _gen(seed: int, device):
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def grf(shape, slope: float, std: float, seed: int, device="cuda"):
    """Gaussian random field with power spectrum |k|^slope, P(0) = 0 (float32).

    Drawn periodic on the next power-of-two grid and cropped to ``shape``, so
    that the FFT plans are of a few power-of-two sizes (an FFT of an awkward
    size would compile a kernel at run time for every new shape)."""
    import torch
    full = tuple(1 << max(0, (int(n) - 1).bit_length()) for n in shape)
    g = _gen(seed, device)
    white = torch.randn(full, generator=g, device=device, dtype=torch.float32)
    spec = torch.fft.rfftn(white)
    del white
    k2 = None
    for ax, n in enumerate(full):
        f = torch.fft.rfftfreq(n, device=device) if ax == len(full) - 1 else torch.fft.fftfreq(n, device=device)
        sh = [1] * len(full)
        sh[ax] = f.numel()
        t = (f * f).reshape(sh)
        k2 = t if k2 is None else k2 + t
    amp = k2.expand(spec.shape).clone()
    amp.view(-1)[0] = 1.0
    amp.pow_(slope / 4.0)
    amp.view(-1)[0] = 0.0
    spec *= amp
    del amp
    field = torch.fft.irfftn(spec, s=full)
    del spec
    field = field[tuple(slice(0, int(n)) for n in shape)].contiguous()
    field -= field.mean(dtype=torch.float64).float()
    field *= std / field.std().item()
    return field


def climate2d(shape, seed: int, dtype=None, device="cuda"):
    """280 - 30 sin^2(lat) + k^-2.5 field (std 5) + 1% of points offset by U[-50, 50]."""
    import torch
    ny, nx = shape
    lat = torch.deg2rad(-90.0 + (torch.arange(ny, device=device, dtype=torch.float64) + 0.5) * 180.0 / ny)[:, None]
    out = (280.0 - 30.0 * torch.sin(lat) ** 2) + grf(shape, -2.5, 5.0, seed, device).double()
    g = _gen(seed + 1, device)
    n = ny * nx
    nsp = max(1, n // 100)
    idx = torch.randperm(n, generator=g, device=device)[:nsp]
    out.view(-1)[idx] += torch.rand(nsp, generator=g, device=device, dtype=torch.float64) * 100.0 - 50.0
    return out.to(dtype or torch.float32)


def smooth3d(shape, seed: int, dtype=None, device="cuda"):
    """8 random Gaussians (amplitude U[0.5,2], width U[4,16]) + separable sines + N(0, 1e-3)."""
    import torch
    g = _gen(seed, device)
    nz, ny, nx = shape
    z = torch.arange(nz, device=device, dtype=torch.float32)[:, None, None]
    y = torch.arange(ny, device=device, dtype=torch.float32)[None, :, None]
    x = torch.arange(nx, device=device, dtype=torch.float32)[None, None, :]
    prm = torch.rand(8, 5, generator=g, device=device, dtype=torch.float64).cpu().tolist()
    out = torch.zeros(shape, device=device, dtype=torch.float32)
    for a, w, cz, cy, cx in prm:
        a = 0.5 + 1.5 * a
        w = 4.0 + 12.0 * w
        cz, cy, cx = cz * nz, cy * ny, cx * nx
        # separable Gaussian: product of three 1D factors
        out += a * (torch.exp(-(z - cz) ** 2 / (2 * w * w)) * torch.exp(-(y - cy) ** 2 / (2 * w * w))
                    * torch.exp(-(x - cx) ** 2 / (2 * w * w)))
    out += torch.sin(0.1 * x) * torch.cos(0.07 * y) * torch.sin(0.05 * z)
    out += torch.randn(shape, generator=g, device=device, dtype=torch.float32) * 1e-3
    return out.to(dtype or torch.float32)


def cosmo3d(shape, seed: int, device="cuda"):
    """Lognormal density exp(g), g a k^-3 Gaussian random field of std 1.5 (float32)."""
    return grf(shape, -3.0, 1.5, seed, device).exp_()


def sines3d(shape, device="cuda"):
    """sin(0.1x) cos(0.07y) sin(0.05z) on integer indices (x fastest): the
    separable component of the small-case recipe, without Gaussians or noise."""
    import torch
    nz, ny, nx = shape
    z = torch.arange(nz, device=device, dtype=torch.float64)[:, None, None]
    y = torch.arange(ny, device=device, dtype=torch.float64)[None, :, None]
    x = torch.arange(nx, device=device, dtype=torch.float64)[None, None, :]
    return (torch.sin(0.1 * x) * torch.cos(0.07 * y) * torch.sin(0.05 * z)).float().contiguous()


def velocity3d(shape, seed: int, device="cuda"):
    """Zero-mean velocity-like k^-3 Gaussian random field of std 300 (float32)."""
    return grf(shape, -3.0, 300.0, seed, device)


def batch_field(spec, device="cuda"):
    """A field of ``fieldgen.batch_fields`` made on the device."""
    if spec["kind"] == "climate2d":
        return climate2d(spec["shape"], spec["seed"], device=device)
    return smooth3d(spec["shape"], spec["seed"], device=device)


def request_field(req, device="cuda"):
    """Field data of a ``fieldgen.request_stream`` request made on the device,
    with the recipe of ``fieldgen.request_field``: a random walk plus a slow
    sine in 1D, 280 + 10 sin(0.01y) cos(0.013x) + N(0, 0.05) in 2D, and
    sin(0.05x) cos(0.04y) sin(0.03z) + N(0, 1e-3) in 3D."""
    import torch
    shape, sd = req["shape"], req["seed"]
    import numpy as np
    dt = torch.float32 if np.dtype(req["dtype"]) == np.float32 else torch.float64
    g = _gen(sd, device)
    if len(shape) == 1:
        n = shape[0]
        xs = torch.arange(n, device=device, dtype=torch.float64)
        f = torch.sin(xs * 0.001) * 10 + torch.cumsum(torch.randn(n, generator=g, device=device,
                                                                   dtype=torch.float64) * 0.05, 0)
        return f.to(dt)
    if len(shape) == 2:
        ny, nx = shape
        yy = torch.arange(ny, device=device, dtype=torch.float64)[:, None]
        xx = torch.arange(nx, device=device, dtype=torch.float64)[None, :]
        f = 280 + 10 * torch.sin(yy * 0.01) * torch.cos(xx * 0.013)
        f = f.to(dt) + torch.randn(shape, generator=g, device=device, dtype=dt) * 0.05
        return f
    nz, ny, nx = shape
    zz = torch.arange(nz, device=device, dtype=dt)[:, None, None]
    yy = torch.arange(ny, device=device, dtype=dt)[None, :, None]
    xx = torch.arange(nx, device=device, dtype=dt)[None, None, :]
    f = torch.sin(0.05 * xx) * torch.cos(0.04 * yy) * torch.sin(0.03 * zz)
    f += torch.randn(shape, generator=g, device=device, dtype=dt) * 1e-3
    return f
