"""The C-ABI entry points beyond compress/decompress (MI355X only).

* sz_compress_async: eager, and captured into a HIP graph (torch's graph
  capture of the library's launches on the capturing stream) and replayed
  several times with other device work and host synchronisations between
  the replays; every replay is checked against the eager result, the size
  and status it writes to device memory, sz_compress and the oracle.
* sz_ctx_create / sz_ctx_destroy: contexts made and destroyed in turn (and
  several alive at once) give identical results; destroying NULL is a no-op.
* sz_ctx_profile: a stage mask times only the stages it names; values it
  does not define are rejected.
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


def _bufs(Z, p):
    import torch
    cap = Z.sz_compress_bound(p)
    out = torch.zeros(cap, dtype=torch.uint8, device="cuda")
    size = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    status = torch.full((1,), 777, dtype=torch.int32, device="cuda")
    return cap, out, size, status


def test_async_eager_matches_sync_and_oracle(Z, oracle):
    import torch
    kw = dict(layers=1, m=8, eb_mode="rel", eb_rel=1e-4)
    for shape in ((40, 50, 60), (300, 257), (10000,)):
        xh = F.smooth3d(shape) if len(shape) == 3 else (F.climate2d(shape) if len(shape) == 2 else
                                                        np.cumsum(F.rng(1).normal(0, 1, shape[0])).astype(np.float32))
        x = torch.from_numpy(xh).cuda()
        p = Z.make_params(shape, "float32", **kw)
        cap, out, size, status = _bufs(Z, p)
        st = torch.cuda.current_stream()
        rc = Z.sz_compress_async(Z.context(0), p, x.data_ptr(), out.data_ptr(), cap, size.data_ptr(),
                                 status.data_ptr(), st.cuda_stream)
        assert rc == 0
        st.synchronize()
        assert int(status.item()) == 0
        n = int(size.item())
        ref, _ = oracle.compress(xh, **kw)
        comp, _ = Z.compress(x, **kw)
        assert n == len(ref) == comp.numel()
        assert out[:n].cpu().numpy().tobytes() == ref == comp.cpu().numpy().tobytes()


def test_async_capacity_status_on_device(Z):
    import torch
    x = torch.from_numpy(F.smooth3d((24, 32, 40))).cuda()
    p = Z.make_params(tuple(x.shape), "float32", layers=1, m=8, eb_mode="rel", eb_rel=1e-4)
    out = torch.zeros(1000, dtype=torch.uint8, device="cuda")
    size = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    status = torch.full((1,), 777, dtype=torch.int32, device="cuda")
    st = torch.cuda.current_stream()
    rc = Z.sz_compress_async(Z.context(0), p, x.data_ptr(), out.data_ptr(), 1000, size.data_ptr(),
                             status.data_ptr(), st.cuda_stream)
    assert rc == 0  # nothing is known on the host; the device reports it
    st.synchronize()
    assert int(status.item()) == Z.SZ_ECAPACITY and int(size.item()) == 0


def test_async_graph_capture_and_replays(Z, oracle):
    import torch
    shape = (48, 64, 80)
    kw = dict(layers=1, m=8, eb_mode="rel", eb_rel=1e-4)
    fields = [F.smooth3d(shape, seed=F.BASE_SEED + 60 + i) for i in range(3)]
    x = torch.from_numpy(fields[0]).cuda()
    p = Z.make_params(shape, "float32", **kw)
    cap, out, size, status = _bufs(Z, p)
    ctx = Z.context(0)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        # eager call first: the context's scratch is sized before the capture
        assert Z.sz_compress_async(ctx, p, x.data_ptr(), out.data_ptr(), cap, size.data_ptr(), status.data_ptr(),
                                   side.cuda_stream) == 0
    side.synchronize()
    eager0 = out[:int(size.item())].cpu().numpy().tobytes()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        rc = Z.sz_compress_async(ctx, p, x.data_ptr(), out.data_ptr(), cap, size.data_ptr(), status.data_ptr(),
                                 torch.cuda.current_stream().cuda_stream)
    assert rc == 0
    other = Z.sz_ctx_create(0)  # eager work between replays on its own context
    try:
        for rep in range(4):
            xi = fields[rep % 3]
            print(f"[graph] replay {rep}", file=sys.stderr, flush=True)
            x.copy_(torch.from_numpy(xi).cuda())
            out.fill_(0)
            size.fill_(-1)
            status.fill_(777)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert int(status.item()) == 0
            got = out[:int(size.item())].cpu().numpy().tobytes()
            ref, _ = oracle.compress(xi, **kw)
            assert got == ref, f"replay {rep}"
            if rep == 0:
                assert got == eager0
            # unrelated eager device work and a second context in between
            y = torch.from_numpy(F.climate2d((100, 120))).cuda()
            pc = Z.make_params((100, 120), "float32", **kw)
            ob = torch.empty(Z.sz_compress_bound(pc), dtype=torch.uint8, device="cuda")
            rc2, n2, _ = Z.sz_compress(other, pc, y.data_ptr(), ob.data_ptr(), ob.numel(),
                                       torch.cuda.current_stream().cuda_stream)
            assert rc2 == 0 and n2 > 0
            (y * 2).sum().item()
    finally:
        Z.sz_ctx_destroy(other)
    del g


def test_ctx_create_destroy(Z, oracle):
    import torch
    xh = F.climate2d((200, 300))
    x = torch.from_numpy(xh).cuda()
    kw = dict(layers=2, m=0, eb_mode="rel", eb_rel=1e-4)
    ref, _ = oracle.compress(xh, **kw)
    p = Z.make_params(xh.shape, "float32", **kw)
    cap = Z.sz_compress_bound(p)
    out = torch.empty(cap, dtype=torch.uint8, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    alive = []
    for i in range(6):
        c = Z.sz_ctx_create(0)
        rc, n, _ = Z.sz_compress(c, p, x.data_ptr(), out.data_ptr(), cap, st)
        assert rc == 0 and out[:n].cpu().numpy().tobytes() == ref
        if i % 2:
            Z.sz_ctx_destroy(c)
        else:
            alive.append(c)
    for c in alive:
        rc, n, _ = Z.sz_compress(c, p, x.data_ptr(), out.data_ptr(), cap, st)
        assert rc == 0 and out[:n].cpu().numpy().tobytes() == ref
        Z.sz_ctx_destroy(c)
    Z.sz_ctx_destroy(0)  # NULL: no-op


def test_stage_profiler_mask(Z):
    """sz_ctx_profile with a stage mask times only those stages; bad values
    are rejected."""
    import torch
    ctx = Z.sz_ctx_create(0)
    try:
        x = torch.from_numpy(F.smooth3d((48, 40, 72))).cuda()
        p = Z.make_params(tuple(x.shape), x.dtype, layers=1, m=8, eb_mode="rel", eb_rel=1e-4)
        cap = Z.sz_compress_bound(p)
        comp = torch.empty(cap, dtype=torch.uint8, device="cuda")
        out = torch.empty_like(x)
        st_ = torch.cuda.current_stream().cuda_stream

        def roundtrip():
            rc, size, _ = Z.sz_compress(ctx, p, x.data_ptr(), comp.data_ptr(), cap, st_)
            assert rc == 0
            assert Z.sz_decompress(ctx, comp.data_ptr(), size, out.data_ptr(), x.numel() * 4, st_) == 0

        assert Z.sz_ctx_profile(ctx, True, stages=("sweep_compress", "sweep_decompress")) == 0
        roundtrip()
        prof = Z.sz_ctx_profile_read(ctx)
        timed = {k for k, (ms, calls) in prof.items() if calls}
        assert timed == {"sweep_compress", "sweep_decompress"}, prof
        assert Z.sz_ctx_profile(ctx, True) == 0
        roundtrip()
        prof = Z.sz_ctx_profile_read(ctx)
        assert {"range", "sweep_compress", "encode", "decode", "sweep_decompress"} <= \
            {k for k, (ms, calls) in prof.items() if calls}
        assert Z.sz_ctx_profile(ctx, False) == 0
        roundtrip()
        assert all(calls == 0 for ms, calls in Z.sz_ctx_profile_read(ctx).values())
        L = Z.lib()
        import ctypes as C
        for bad in (2, 0x20000, -1, 0x10000 | 0x20000):
            assert L.sz_ctx_profile(C.c_void_p(ctx), bad) == -1, bad
    finally:
        Z.sz_ctx_destroy(ctx)
