"""Served form (MI355X only): continuous batching of compress / decompress
requests under an HBM budget.

Every result must equal the result of the same request run alone through
sz_compress / sz_decompress (container bytes, decompressed bits), whatever
else is in flight; admission must respect the workspace pool and overlap
requests on the device.
"""
import threading

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


def _bits(t):
    a = t.cpu().numpy()
    return a.view(np.uint32 if a.dtype == np.float32 else np.uint64)


def request_mix(count=18, seed=5):
    """Requests shaped like the served workload, at test sizes."""
    reqs = F.request_stream(rate=1000.0, duration=1.0, seed=F.BASE_SEED + seed, size_scale=1 / 64,
                            max_bytes=64 << 20, min_bytes=1 << 20)[:count]
    return reqs


def test_server_results_equal_alone(Z):
    import torch
    reqs = request_mix()
    assert len(reqs) >= 12
    data = [dev(F.request_field(r)) for r in reqs]
    kws = [dict(layers=1, m=8, eb_mode="rel", eb_rel=r["eb_rel"]) for r in reqs]
    # alone: every compress, and the containers the decompress requests use
    alone = [Z.compress(x, **kw)[0].clone() for x, kw in zip(data, kws)]
    alone_dec = [Z.decompress(c) for c in alone]
    torch.cuda.synchronize()
    # a budget that holds a few workspaces at once, not all
    srv = Z.Server(hbm_budget=256 << 20, slots=4)
    ids, outs = [], []
    for r, x, kw, c in zip(reqs, data, kws, alone):
        if r["op"] == "compress":
            out = torch.zeros(Z.sz_compress_bound(Z.make_params(tuple(x.shape), x.dtype, **kw)), dtype=torch.uint8,
                              device="cuda")
            ids.append(srv.submit_compress(x, out, **kw))
        else:
            out = torch.zeros_like(x)
            ids.append(srv.submit_decompress(c, out))
        outs.append(out)
    for i, (r, rid) in enumerate(zip(reqs, ids)):
        res = srv.wait(rid, timeout_ms=120000)
        assert res["status"] == 0, (i, res)
        assert res["t_submit"] <= res["t_admit"] <= res["t_done"]
        if r["op"] == "compress":
            got = outs[i][: res["out_size"]].cpu().numpy().tobytes()
            assert got == alone[i].cpu().numpy().tobytes(), f"request {i} {r['shape']} {r['dtype']}"
        else:
            assert res["out_size"] == data[i].numel() * data[i].element_size()
            assert np.array_equal(_bits(outs[i]), _bits(alone_dec[i])), f"request {i} {r['shape']} {r['dtype']}"
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["in_flight"] == 0
    assert st["max_in_flight"] >= 2, st
    assert st["pool_peak_bytes"] <= st["pool_bytes"]
    srv.close()


def test_server_threads_and_headers(Z):
    """Submissions from several host threads; decompress with host headers."""
    import torch
    xs = [dev(F.smooth3d((20 + 3 * i, 40, 33), seed=60 + i)) for i in range(6)]
    comps = [Z.compress(x, layers=1, m=8, eb_mode="rel", eb_rel=1e-4)[0].clone() for x in xs]
    ref = [Z.decompress(c) for c in comps]
    torch.cuda.synchronize()
    srv = Z.Server(hbm_budget=64 << 20, slots=3)
    results = [None] * len(xs)
    outs = [torch.zeros_like(x) for x in xs]

    def worker(i):
        hdr = comps[i][:192].cpu().numpy().tobytes()
        rid = srv.submit_decompress(comps[i], outs[i], header=hdr)
        results[i] = srv.wait(rid, timeout_ms=60000)

    th = [threading.Thread(target=worker, args=(i,)) for i in range(len(xs))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for i in range(len(xs)):
        assert results[i]["status"] == 0
        assert np.array_equal(_bits(outs[i]), _bits(ref[i]))
    srv.close()


def test_server_errors(Z):
    import torch
    srv = Z.Server(hbm_budget=4 << 20, slots=2)
    x = dev(F.smooth3d((64, 64, 64), seed=70))
    big = torch.zeros(Z.sz_compress_bound(Z.make_params(tuple(x.shape), x.dtype, m=8, eb_mode="rel", eb_rel=1e-4)),
                      dtype=torch.uint8, device="cuda")
    # workspace of a 64^3 field exceeds a 4 MiB pool
    rid = srv.submit_compress(x, big, m=8, eb_mode="rel", eb_rel=1e-4)
    assert srv.wait(rid, 60000)["status"] == Z.SZ_ENOMEM
    # a corrupt container
    bad = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    rid = srv.submit_decompress(bad, torch.zeros(16, device="cuda"))
    assert srv.wait(rid, 60000)["status"] == Z.SZ_ECORRUPT
    # capacity too small for the output
    small = dev(F.smooth3d((8, 8, 8), seed=71))
    c = Z.compress(small, m=8, eb_mode="rel", eb_rel=1e-4)[0].clone()
    rid = srv.submit_decompress(c, torch.zeros(16, device="cuda"))
    assert srv.wait(rid, 60000)["status"] == Z.SZ_ECAPACITY
    rc, _ = Z.sz_server_wait(srv.handle, 987654, 10)
    assert rc == Z.SZ_EINVAL
    srv.close()
    # the footprint counts input and output as well as the workspace: a 1D
    # field whose workspace alone fits the budget but whose input, output
    # capacity and workspace together do not is refused
    srv = Z.Server(hbm_budget=16 << 20, slots=2)
    w = dev(np.cumsum(np.random.default_rng(72).normal(0, 1, 1 << 20)).astype(np.float32))
    ob = torch.zeros(Z.sz_compress_bound(Z.make_params(tuple(w.shape), w.dtype, m=8, eb_mode="rel", eb_rel=1e-4)),
                     dtype=torch.uint8, device="cuda")
    rid = srv.submit_compress(w, ob, m=8, eb_mode="rel", eb_rel=1e-4)
    res = srv.wait(rid, 60000)
    assert res["status"] == 0 and res["workspace_bytes"] < (16 << 20) - 8 * (1 << 20)
    w2 = dev(np.cumsum(np.random.default_rng(73).normal(0, 1, 3 << 20)).astype(np.float32))
    ob2 = torch.zeros(Z.sz_compress_bound(Z.make_params(tuple(w2.shape), w2.dtype, m=8, eb_mode="rel",
                                                        eb_rel=1e-4)), dtype=torch.uint8, device="cuda")
    rid = srv.submit_compress(w2, ob2, m=8, eb_mode="rel", eb_rel=1e-4)
    res = srv.wait(rid, 60000)
    assert res["status"] == Z.SZ_ENOMEM and res["workspace_bytes"] < (16 << 20)
    srv.close()
