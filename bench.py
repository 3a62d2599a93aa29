"""Benchmark of the compressor's hot path on one MI355X.

One step = compress + decompress of a 512^3 float32 lognormal density field
(the cosmology-like workload: exp of a Gaussian random field with spectrum
k^-3, std 1.5), 1-layer prediction, value-range-relative bound 1e-4, m = 8
(256 codes), through the C ABI with the field already resident in HBM.

Prints ONE JSON line: compress+decompress GB/s (2S / (t_c + t_d)), the
fraction of HBM peak of the algorithmic bytes, the roofline of the dominant
kernel (algorithmic bytes per launch / its HIP-event duration), and the CPU
oracle timed on a bounded sample of the same field.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "compress+decompress GB/s on 512^3 FP32 @ eb=1e-4·range, %HBM peak; p99 latency served"
HBM_PEAK_GBPS = 8000.0
HEADER = 192


def sweep_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("sweep.hpp", "common.hpp"):
        with open(os.path.join(ROOT, "paper_1706_03791_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str, n_launch_bytes: float):
    """HBM bytes of the dominant kernel from committed rocprofv3 PMC runs,
    valid only while the kernel source is unchanged."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_hash") != sweep_source_hash():
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(x: np.ndarray, planes: int, kw: dict):
    import oracle as O
    sample = np.ascontiguousarray(x[:planes])
    t0 = time.perf_counter()
    buf, st = O.compress(sample, **kw)
    t1 = time.perf_counter()
    out = O.decompress(buf)
    t2 = time.perf_counter()
    assert out.shape == sample.shape
    gbps = 2 * sample.nbytes / ((t1 - t0) + (t2 - t1)) / 1e9
    return {"value": round(gbps, 6), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"first {planes} z-planes of the same field ({sample.shape[0]}x{sample.shape[1]}x"
                      f"{sample.shape[2]} f32, {sample.nbytes / 2**20:.0f} MiB): compress "
                      f"{t1 - t0:.2f} s + decompress {t2 - t1:.2f} s, single thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-planes", type=int, default=32)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}); "
              "the single-GPU kernel is the unit a multi-GPU run would shard.", file=sys.stderr)
        sys.exit(2)

    import torch
    import fieldgen as F
    import paper_1706_03791_amd as Z

    n = args.size
    kw = dict(layers=1, m=8, eb_mode="rel", eb_rel=1e-4)
    print(f"[bench] generating {n}^3 field", file=sys.stderr, flush=True)
    x = F.cosmo3d((n, n, n))
    S = x.nbytes
    xd = torch.from_numpy(x).cuda()
    p = Z.make_params(x.shape, "float32", **kw)
    cap = Z.sz_compress_bound(p)
    comp = torch.empty(cap, dtype=torch.uint8, device="cuda")
    out = torch.empty_like(xd)
    ctx = Z.context(0)
    stream = torch.cuda.current_stream().cuda_stream

    def step():
        t0 = time.perf_counter()
        rc, size, st = Z.sz_compress(ctx, p, xd.data_ptr(), comp.data_ptr(), cap, stream)
        t1 = time.perf_counter()
        if rc:
            raise Z.SzError(rc, "sz_compress")
        rc = Z.sz_decompress(ctx, comp.data_ptr(), size, out.data_ptr(), out.numel() * 4, stream)
        t2 = time.perf_counter()
        if rc:
            raise Z.SzError(rc, "sz_decompress")
        return t1 - t0, t2 - t1, size, st

    print("[bench] warmup", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    Z.sz_ctx_profile(ctx, True)
    torch.cuda.synchronize()
    tc, td = [], []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        a, b, size, st = step()
        tc.append(a)
        td.append(b)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    prof = Z.sz_ctx_profile_read(ctx)
    Z.sz_ctx_profile(ctx, False)
    print(f"[bench] timed {args.steps} steps in {t_total:.3f} s", file=sys.stderr, flush=True)

    # correctness guard on the last step: the bound holds everywhere
    err = (out.double() - xd.double()).abs().max().item()
    assert err < st.eb_used, (err, st.eb_used)

    Cb = size
    t_c, t_d = float(np.mean(tc)), float(np.mean(td))
    value = 2 * S / (t_c + t_d) / 1e9
    alg_bytes = (2 * S + Cb) + (Cb + S)
    hbm_frac = alg_bytes / (t_c + t_d) / 1e9 / HBM_PEAK_GBPS

    # dominant kernel stage and its algorithmic bytes per launch
    per_call = {k: (ms / calls if calls else 0.0) for k, (ms, calls) in prof.items()}
    alg_per_stage = {"range": S, "sweep_compress": S, "encode": Cb, "decode": Cb,
                     "sweep_decompress": S, "unpred": 0, "dectab": 0, "codebook": 0}
    dom = max(("sweep_compress", "sweep_decompress", "encode", "decode", "range"), key=lambda k: per_call[k])
    dom_ms = per_call[dom]
    achieved = alg_per_stage[dom] / (dom_ms / 1e3) / 1e9
    traffic = load_traffic(dom, f"cosmo{n}", alg_per_stage[dom])

    res = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_total / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"cosmo3d {n}^3 f32 lognormal density (GRF k^-3, std 1.5), 1-layer, "
                               f"m=8, eb_rel=1e-4, compress+decompress", "n_points": int(x.size),
                   "field_bytes": int(S)},
        "compress_GBps": round(S / t_c / 1e9, 3),
        "decompress_GBps": round(S / t_d / 1e9, 3),
        "hbm_frac": round(hbm_frac, 4),
        "compression_factor": round(S / Cb, 3),
        "hit_rate": st.hit_rate,
        "n_unpred": int(st.n_unpred),
        "stage_ms": {k: round(v, 4) for k, v in per_call.items()},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 2),
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic,
                     "algorithmic_bytes_per_launch": int(alg_per_stage[dom]),
                     "launch_ms": round(dom_ms, 4)},
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(x, args.cpu_planes, kw)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
