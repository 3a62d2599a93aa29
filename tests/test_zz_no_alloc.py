"""The entry point that allocates nothing, against the one it mirrors (MI355X).

sz_compress_async_noalloc runs the pipeline of sz_compress_async with its
workspace in the library's static per-device scratch.  Two calls in a row,
the second on a smaller field (so it reuses scratch the first left dirty),
must each give the bytes, size and status of sz_compress_async on the same
input, and those bytes must equal the oracle's.  A field whose workspace
exceeds the static scratch is refused before anything is enqueued.
"""
import sys

import numpy as np
import pytest

import fieldgen as F

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Z():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    import paper_1706_03791_amd as Z
    Z.lib()
    return Z


def _run(Z, fn, x, kw):
    import torch
    p = Z.make_params(tuple(x.shape), x.dtype, **kw)
    cap = Z.sz_compress_bound(p)
    out = torch.full((cap,), 0xA5, dtype=torch.uint8, device=x.device)
    size = torch.full((1,), -1, dtype=torch.int64, device=x.device)
    status = torch.full((1,), 12345, dtype=torch.int32, device=x.device)
    stream = torch.cuda.current_stream()
    rc = fn(Z.context(0), p, x.data_ptr(), out.data_ptr(), cap, size.data_ptr(), status.data_ptr(),
            stream.cuda_stream)
    assert rc == 0, Z.strerror(rc)
    stream.synchronize()
    n, s = int(size.item()), int(status.item())
    return out[:n].cpu().numpy().tobytes(), n, s


CASES = [
    ("smooth 96x100x110 f32", lambda: F.smooth3d((96, 100, 110)), dict(layers=1, m=8, eb_mode="rel", eb_rel=1e-4)),
    ("climate 300x500 f32 adaptive m", lambda: F.climate2d((300, 500)),
     dict(layers=1, m=0, eb_mode="rel", eb_rel=1e-5)),
    ("walk 20000 f64 2 layers", lambda: np.cumsum(F.rng(9).normal(0, 1, 20000)),
     dict(layers=2, m=12, eb_mode="abs", eb_abs=1e-3)),
]


def test_noalloc_matches_async_two_calls(Z, oracle):
    import torch
    # the largest field first, then smaller ones over the scratch it left
    for name, make, kw in (CASES[0], CASES[1], CASES[2], CASES[1]):
        print(f"[noalloc] {name}", file=sys.stderr, flush=True)
        xh = np.ascontiguousarray(make())
        x = torch.from_numpy(xh).cuda()
        got, n, s = _run(Z, Z.sz_compress_async_noalloc, x, kw)
        want, n0, s0 = _run(Z, Z.sz_compress_async, x, kw)
        assert (s, s0) == (0, 0)
        assert n == n0 and got == want, name
        ref, _ = oracle.compress(xh, **kw)
        assert got == ref, name


def test_noalloc_refuses_fields_beyond_scratch(Z):
    import torch
    p = Z.make_params((1024, 1024, 1024), "float32", layers=1, m=8, eb_mode="rel", eb_rel=1e-4)
    buf = torch.zeros(64, dtype=torch.uint8, device="cuda")
    d = torch.zeros(2, dtype=torch.int64, device="cuda")
    rc = Z.sz_compress_async_noalloc(Z.context(0), p, buf.data_ptr(), buf.data_ptr(), 64, d.data_ptr(),
                                     d.data_ptr() + 8, torch.cuda.current_stream().cuda_stream)
    assert rc == Z.SZ_ESCRATCH
    assert "static" in Z.strerror(rc)
    # the entry point still works after the refusal
    x = torch.from_numpy(F.smooth3d((20, 30, 40))).cuda()
    kw = dict(layers=1, m=8, eb_mode="rel", eb_rel=1e-4)
    got, _, s = _run(Z, Z.sz_compress_async_noalloc, x, kw)
    want, _, _ = _run(Z, Z.sz_compress_async, x, kw)
    assert s == 0 and got == want
