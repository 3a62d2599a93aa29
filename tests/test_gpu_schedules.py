"""Schedule invariance of the single-field sweeps (MI355X only): the race
check of the inter-tile exchange.

Algorithm 1 predicts every point from decompressed neighbours, so the sweep
tiles hand boundary values to each other: as tagged records that the next
tile polls (wave tiles) or behind progress flags (row-per-thread tiles).
Running the same field under different tile shapes (wave tiles or
row-per-thread tiles) and different tile claim orders (another dependence
order inside each block; independent blocks reversed) changes which
workgroup runs which tile, when, and next to whom -- a missing wait or a
stale read shows up as different bytes.  Every schedule must give the
container and the decompressed bits of the default one, which equal the
oracle's.
"""
import sys

import numpy as np
import pytest

import fieldgen as F

pytestmark = pytest.mark.gpu

SCHEDULES = [(0, 0), (0, 1), (0, 2), (1, 0), (1, 1), (1, 2)]


@pytest.fixture(scope="module")
def Z():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    import paper_1706_03791_amd as Z
    Z.lib()
    return Z


def _u(a):
    return a.view(np.uint32 if a.dtype == np.float32 else np.uint64)


CASES = [
    ("smooth 70x150x200 f32", lambda: F.smooth3d((70, 150, 200)), dict(layers=1, m=8, eb_mode="rel", eb_rel=1e-4)),
    ("smooth 40x130x90 f64 blocks", lambda: F.smooth3d((40, 130, 90), dtype=np.float64),
     dict(layers=1, m=0, eb_mode="rel", eb_rel=1e-8, block=(20, 65, 90))),
    ("climate 700x900 f32 2 layers", lambda: F.climate2d((700, 900)), dict(layers=2, m=0, eb_mode="rel", eb_rel=1e-5)),
    ("climate 1000x1300 f32 blocks", lambda: F.climate2d((1000, 1300)),
     dict(layers=1, m=8, eb_mode="rel", eb_rel=1e-4, block=(500, 650))),
    ("walk 300000 f32", lambda: np.cumsum(F.rng(4).normal(0, 1, 300000)).astype(np.float32),
     dict(layers=1, m=8, eb_mode="rel", eb_rel=1e-5)),
]


@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
def test_every_schedule_gives_the_same_bytes(Z, oracle, case):
    import torch
    name, make, kw = CASES[case]
    xh = np.ascontiguousarray(make())
    ref, sref, _, xp = oracle.compress(xh, debug=True, **kw)
    x = torch.from_numpy(xh).cuda()
    ctx = Z.sz_ctx_create(0)  # a context of its own: the schedule is a context setting
    try:
        p = Z.make_params(xh.shape, xh.dtype, **kw)
        cap = Z.sz_compress_bound(p)
        comp = torch.empty(cap, dtype=torch.uint8, device="cuda")
        out = torch.empty_like(x)
        st = torch.cuda.current_stream().cuda_stream
        for sched, claim in SCHEDULES:
            print(f"[schedules] {name}: schedule {sched} claim {claim}", file=sys.stderr, flush=True)
            assert Z.sz_ctx_debug_sweep(ctx, sched, claim) == 0
            for rep in range(2):
                rc, n, _ = Z.sz_compress(ctx, p, x.data_ptr(), comp.data_ptr(), cap, st)
                assert rc == 0
                got = comp[:n].cpu().numpy().tobytes()
                assert got == ref, f"{name}: schedule {sched} claim {claim} rep {rep}: container differs"
                out.fill_(0)
                assert Z.sz_decompress(ctx, comp.data_ptr(), n, out.data_ptr(), out.numel() * out.element_size(),
                                       st) == 0
                want = xh if sref["raw_fallback"] else xp
                assert np.array_equal(_u(out.cpu().numpy()), _u(want)), f"{name}: schedule {sched} claim {claim}"
        assert Z.sz_ctx_debug_sweep(ctx, 2, 0) == Z.SZ_EINVAL
        assert Z.sz_ctx_debug_sweep(ctx, 0, 3) == Z.SZ_EINVAL
    finally:
        Z.sz_ctx_destroy(ctx)
