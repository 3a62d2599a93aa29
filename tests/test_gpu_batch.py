"""Batched form (MI355X only): one batched launch per stage and one persistent
sweep over the tiles of every field, captured into a HIP graph.

The container of every field must be byte-identical to the single-field
path's (itself bit-exact with the oracle, see test_gpu_parity.py) under every
tile schedule, in eager and graph mode, on graph replays, and for a few
fields directly against the oracle.
"""
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


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def single(Z, xs, kws):
    return [bytes(Z.compress(x, **kw)[0].cpu().numpy().tobytes()) for x, kw in zip(xs, kws)]


def batch_bytes(B, xs, use_graph):
    return [bytes(c.cpu().numpy().tobytes()) for c in B.compress(xs, use_graph=use_graph)]


def small_mix(count=10, scale=0.08):
    specs = F.batch_fields(count=count, scale=scale)
    xs = [F.make_batch_field(s) for s in specs]
    kws = [dict(layers=1, m=8, eb_mode="rel", eb_rel=s["eb_rel"]) for s in specs]
    return xs, kws


@pytest.mark.parametrize("schedule", [0, 1, 2, 3])
def test_batch_equals_single_every_schedule(Z, schedule):
    xs, kws = small_mix()
    xd = [dev(x) for x in xs]
    ref = single(Z, xd, kws)
    B = Z.Batch([x.shape for x in xs], "float32", kws, schedule=schedule)
    for use_graph in (False, True):
        got = batch_bytes(B, xd, use_graph)
        for i, (g, r) in enumerate(zip(got, ref)):
            assert g == r, f"field {i} shape {xs[i].shape} schedule {schedule} graph {use_graph}"
    B.close()


def test_batch_autotune_and_replays(Z):
    import torch
    xs, kws = small_mix(count=16, scale=0.1)
    xd = [dev(x) for x in xs]
    ref = single(Z, xd, kws)
    B = Z.Batch([x.shape for x in xs], "float32", kws, schedule=-1)
    for rep in range(4):
        got = batch_bytes(B, xd, True)
        assert got == ref, f"graph replay {rep}"
        # eager work of the program itself between replays
        y = torch.randn(1 << 20, device="cuda")
        torch.cuda.synchronize()
        assert torch.isfinite(y.sum()).item()
    sched, tiles, threads, ms = B.info()
    assert 0 <= sched < 4 and tiles > 0 and threads in (256, 512)
    assert all(t > 0 for t in ms), ms
    assert ms[sched] == min(ms)
    B.close()


def test_batch_mixed_dims_modes(Z):
    """1D/2D/3D, adaptive m (16-bit codes), m = 12, two layers (own sweep
    launches), absolute and combined bounds, blocks, a constant field."""
    g = np.random.default_rng(7)
    xs = [F.smooth3d((20, 70, 33), seed=11),
          F.climate2d((130, 257), seed=12),
          np.cumsum(g.normal(0, 1, 5000)).astype(np.float32),
          F.smooth3d((17, 65, 29), seed=13),
          F.climate2d((64, 64), seed=14),
          np.full((9, 40, 40), 3.25, np.float32),
          F.smooth3d((40, 100, 60), seed=15)]
    kws = [dict(layers=1, m=0, eb_mode="rel", eb_rel=1e-4),
           dict(layers=1, m=12, eb_mode="rel", eb_rel=1e-5),
           dict(layers=1, m=8, eb_mode="abs", eb_abs=1e-2),
           dict(layers=2, m=8, eb_mode="rel", eb_rel=1e-3),
           dict(layers=1, m=8, eb_mode="both", eb_abs=1e-3, eb_rel=1e-4),
           dict(layers=1, m=8, eb_mode="rel", eb_rel=1e-4),
           dict(layers=1, m=8, eb_mode="rel", eb_rel=1e-4, block=(16, 64, 32))]
    xd = [dev(x) for x in xs]
    ref = single(Z, xd, kws)
    for schedule in (0, 2):
        B = Z.Batch([x.shape for x in xs], "float32", kws, schedule=schedule)
        for use_graph in (False, True):
            got = batch_bytes(B, xd, use_graph)
            for i, (a, r) in enumerate(zip(got, ref)):
                assert a == r, f"field {i} shape {xs[i].shape} kw {kws[i]} schedule {schedule} graph {use_graph}"
        B.close()


def test_batch_against_oracle(Z, oracle):
    xs = [F.smooth3d((24, 66, 40), seed=21), F.climate2d((100, 150), seed=22), F.smooth3d((8, 8, 300), seed=23)]
    kws = [dict(layers=1, m=8, eb_mode="rel", eb_rel=1e-4), dict(layers=1, m=8, eb_mode="rel", eb_rel=1e-3),
           dict(layers=1, m=10, eb_mode="abs", eb_abs=1e-4)]
    B = Z.Batch([x.shape for x in xs], "float32", kws, schedule=0)
    got = batch_bytes(B, [dev(x) for x in xs], True)
    for i, (x, kw) in enumerate(zip(xs, kws)):
        ref, _ = oracle.compress(x, **kw)
        assert got[i] == ref, f"field {i}"
    B.close()


def test_batch_f64(Z):
    xs = [F.smooth3d((18, 70, 31), seed=31, dtype=np.float64), F.climate2d((90, 140), seed=32, dtype=np.float64),
          F.smooth3d((33, 20, 50), seed=33, dtype=np.float64)]
    kws = [dict(layers=1, m=8, eb_mode="rel", eb_rel=1e-8), dict(layers=1, m=16, eb_mode="rel", eb_rel=1e-6),
           dict(layers=1, m=8, eb_mode="abs", eb_abs=1e-7)]
    xd = [dev(x) for x in xs]
    ref = single(Z, xd, kws)
    for schedule in (0, 3):
        B = Z.Batch([x.shape for x in xs], "float64", kws, schedule=schedule)
        assert batch_bytes(B, xd, True) == ref
        B.close()


def test_batch_capacity_is_per_field(Z):
    import torch
    xs = [F.smooth3d((16, 64, 40), seed=41), F.smooth3d((16, 64, 40), seed=42)]
    kws = [dict(layers=1, m=8, eb_mode="rel", eb_rel=1e-4)] * 2
    xd = [dev(x) for x in xs]
    params = [Z.make_params(x.shape, "float32", **kw) for x, kw in zip(xs, kws)]
    caps = [Z.sz_compress_bound(p) for p in params]
    caps[1] = 256  # too small for any container of this field
    outs = [torch.zeros(c, dtype=torch.uint8, device="cuda") for c in caps]
    sizes = torch.zeros(2, dtype=torch.int64, device="cuda")
    status = torch.zeros(2, dtype=torch.int32, device="cuda")
    h = Z.sz_batch_create(Z.context(0), params, 1)
    rc = Z.sz_batch_compress(h, [x.data_ptr() for x in xd], [o.data_ptr() for o in outs], caps, sizes.data_ptr(),
                             status.data_ptr(), True, torch.cuda.current_stream().cuda_stream)
    assert rc == 0
    st = status.cpu().tolist()
    assert st[0] == 0 and st[1] == Z.SZ_ECAPACITY, st
    ref = single(Z, xd[:1], kws[:1])[0]
    assert bytes(outs[0][: int(sizes[0])].cpu().numpy().tobytes()) == ref
    Z.sz_batch_destroy(h)
