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
    for f in ("sweep.hpp", "wsweep.hpp", "sweep_launch.hpp", "common.hpp"):
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


# Algorithmic bytes of each stage per launch: what the method itself must
# move there (the range pass reads the field, the prediction sweep reads it,
# the encoder writes the container, the decoder reads it, the reconstruction
# writes the field).  The intermediate code array (one code of w bytes per
# point, written by the sweep and read by the coder, or written by the
# decoder and read by the reconstruction) is design traffic, reported apart.
def stage_bytes(S: int, Cb: int, npts: int, w: int):
    alg = {"range": S, "sweep_compress": S, "encode": Cb, "decode": Cb, "sweep_decompress": S}
    design = {"range": 0, "sweep_compress": npts * w, "encode": npts * w, "decode": npts * w,
              "sweep_decompress": npts * w}
    return alg, design


def stage_roofline(per_call_ms: dict, S: int, Cb: int, npts: int, w: int):
    """Roofline line of the stage with the longest launch: its algorithmic
    bytes per launch over its HIP-event duration, against the HBM peak."""
    alg, design = stage_bytes(S, Cb, npts, w)
    dom = max(alg, key=lambda k: per_call_ms.get(k, 0.0))
    ms = per_call_ms[dom]
    achieved = alg[dom] / (ms / 1e3) / 1e9
    return {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBPS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None,
            "algorithmic_bytes_per_launch": int(alg[dom]), "design_bytes_per_launch": int(design[dom]),
            "launch_ms": round(ms, 4)}


def host_cpus() -> dict:
    """The host's processor as the run sees it."""
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"cpu_model": cpu_model(), "host_cpus": os.cpu_count(), "usable_cpus": usable}


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
                      f"{t1 - t0:.2f} s + decompress {t2 - t1:.2f} s, single thread", **host_cpus()}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return " ".join(line.split(":", 1)[1].split())
    except OSError:
        pass
    return "unknown"


_WORKER = r"""
import json, sys, time
import numpy as np
sys.path.insert(0, sys.argv[1])
import oracle as O
x = np.load(sys.argv[2])
kw = json.loads(sys.argv[3])
t0 = time.perf_counter()
buf, st = O.compress(x, **kw)
t1 = time.perf_counter()
out = O.decompress(buf)
t2 = time.perf_counter()
assert out.shape == x.shape
print(json.dumps({"bytes": int(x.nbytes), "t_c": t1 - t0, "t_d": t2 - t1}))
"""


def cpu_all_cores(x: np.ndarray, planes: int, kw: dict, workers: int):
    """The oracle on every host core at once: one process per core, each
    compressing and decompressing its own slab of `planes` z-planes (the
    paper's model of independent per-process fields).  A different, slab-split
    output: reported beside the single-thread baseline, never used for parity."""
    import shutil
    import subprocess
    import tempfile
    workers = max(1, min(workers, x.shape[0] // planes))
    d = tempfile.mkdtemp(prefix="szcpu_", dir="/tmp")
    try:
        paths = []
        for k in range(workers):
            pth = os.path.join(d, f"slab{k}.npy")
            np.save(pth, np.ascontiguousarray(x[k * planes:(k + 1) * planes]))
            paths.append(pth)
        t0 = time.perf_counter()
        procs = [subprocess.Popen([sys.executable, "-c", _WORKER, ROOT, pth, json.dumps(kw)],
                                  stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True) for pth in paths]
        rows = []
        for pr in procs:
            out, err = pr.communicate(timeout=600)
            if pr.returncode:
                raise RuntimeError(f"oracle worker failed: {err[-500:]}")
            rows.append(json.loads(out.strip().splitlines()[-1]))
        wall = time.perf_counter() - t0
    finally:
        shutil.rmtree(d, ignore_errors=True)
    total = sum(r["bytes"] for r in rows)
    return {"value": round(2 * total / wall / 1e9, 6), "unit": "GB/s", "cores": workers,
            "kind": "oracle, slab-split: one process per core on independent slabs",
            "sample": f"{workers} slabs of {planes} z-planes ({total / 2**20:.0f} MiB in all), compress + "
                      f"decompress each, {wall:.2f} s wall including process start", **host_cpus()}


SWEEP_STAGES = ("sweep_compress", "sweep_decompress")
BREAKDOWN_STEPS = 3


def merge_profiles(every_stage: dict, timed: dict) -> dict:
    """Stage (ms, calls): the timed steps' figures where they were recorded,
    else those of the untimed steps with every stage timed."""
    out = dict(every_stage)
    for k, (ms, calls) in timed.items():
        if calls:
            out[k] = (ms, calls)
    return out


def roundtrip(Z, torch, x, kw, steps=3, warmup=1):
    """Timed compress + decompress of a resident field through the C ABI;
    returns (row dict, reconstruction, stats)."""
    p = Z.make_params(tuple(x.shape), x.dtype, **kw)
    cap = Z.sz_compress_bound(p)
    comp = torch.empty(cap, dtype=torch.uint8, device="cuda")
    out = torch.empty_like(x)
    ctx = Z.context(0)
    st_ = torch.cuda.current_stream().cuda_stream
    S = x.numel() * x.element_size()
    tc, td = [], []
    for i in range(warmup + steps):
        if i == warmup:
            Z.sz_ctx_profile(ctx, True, stages=SWEEP_STAGES)
        t0 = time.perf_counter()
        rc, size, st = Z.sz_compress(ctx, p, x.data_ptr(), comp.data_ptr(), cap, st_)
        t1 = time.perf_counter()
        if rc:
            raise Z.SzError(rc, "sz_compress")
        rc = Z.sz_decompress(ctx, comp.data_ptr(), size, out.data_ptr(), S, st_)
        t2 = time.perf_counter()
        if rc:
            raise Z.SzError(rc, "sz_decompress")
        if i >= warmup:
            tc.append(t1 - t0)
            td.append(t2 - t1)
    prof_timed = Z.sz_ctx_profile_read(ctx)
    Z.sz_ctx_profile(ctx, True)
    for _ in range(min(steps, BREAKDOWN_STEPS)):
        rc, size, st = Z.sz_compress(ctx, p, x.data_ptr(), comp.data_ptr(), cap, st_)
        if rc:
            raise Z.SzError(rc, "sz_compress")
        rc = Z.sz_decompress(ctx, comp.data_ptr(), size, out.data_ptr(), S, st_)
        if rc:
            raise Z.SzError(rc, "sz_decompress")
    prof = merge_profiles(Z.sz_ctx_profile_read(ctx), prof_timed)
    Z.sz_ctx_profile(ctx, False)
    t_c, t_d = float(np.median(tc)), float(np.median(td))
    row = {"GBps": round(2 * S / (t_c + t_d) / 1e9, 3), "compress_GBps": round(S / t_c / 1e9, 3),
           "decompress_GBps": round(S / t_d / 1e9, 3), "compression_factor": round(S / size, 3),
           "bits_per_value": round(8.0 * size / x.numel(), 4), "hit_rate": round(st.hit_rate, 6),
           "m_used": int(st.m_used),
           "stage_ms": {k: round(ms / calls, 4) for k, (ms, calls) in prof.items() if calls}}
    del comp
    return row, out, st


def quality_row(Z, x, xr, eb, max_lag=0):
    """On-device distortion metrics (Sec. II Metrics 2-3, Sec. V autocorrelation)."""
    q = Z.quality(x, xr, max_lag=max_lag)
    row = {"psnr_db": round(q["psnr"], 3), "nrmse": q["nrmse"], "rmse": q["rmse"],
           "pearson": q["pearson"], "max_err_over_eb": round(q["max_abs_err"] / eb, 6)}
    if max_lag:
        row["err_autocorr"] = [round(v, 6) for v in q["autocorr"]]
    return row


def bench_cosmo_extras(Z, torch, n, steps=3):
    """The other two runs of the cosmology workload: the velocity-like field
    (f32, relative bound 1e-4, m = 8) and the density in f64 at a relative
    bound of 1e-8 with the adaptive interval count."""
    import fieldgen as F
    import fieldgen.gpu as G
    out = {}
    runs = (("velocity_f32", lambda: G.velocity3d((n, n, n), F.BASE_SEED + 102), dict(m=8, eb_rel=1e-4)),
            ("density_f64", lambda: G.cosmo3d((n, n, n), F.BASE_SEED + 2).double(), dict(m=0, eb_rel=1e-8)))
    for name, make, extra in runs:
        print(f"[bench] cosmology extra: {name}", file=sys.stderr, flush=True)
        x = make()
        torch.cuda.synchronize()
        kw = dict(layers=1, eb_mode="rel", **extra)
        row, xr, st = roundtrip(Z, torch, x, kw, steps=steps)
        row.update(quality_row(Z, x, xr, st.eb_used))
        row["eb_rel"] = extra["eb_rel"]
        S = x.numel() * x.element_size()
        row["roofline"] = stage_roofline(row["stage_ms"], S, int(round(S / row["compression_factor"])), x.numel(),
                                         1 if st.m_used <= 8 else 2)
        out[name] = row
        del x, xr
        torch.cuda.empty_cache()
    return out


def layer_study(Z, torch, eb_rels=(1e-4,), samples=(None, (900, 1800)), field="climate2d"):
    """Best-layer study (Sec. III-B, Table II): R_PH from decompressed and
    from original neighbours, n = 1..4, on the 1800x3600 climate-like field
    or on the smooth separable-sine 256^3 field."""
    import fieldgen as F
    import fieldgen.gpu as G
    x = G.climate2d((1800, 3600), F.BASE_SEED + 1) if field == "climate2d" else G.sines3d((256, 256, 256))
    rows = []
    for eb in eb_rels:
        for smp in samples:
            r = Z.layer_survey(x, sample=smp, eb_mode="rel", eb_rel=eb)
            rows.append({"field": field, "eb_rel": eb, "sample": list(smp) if smp else list(x.shape),
                         "rph_decomp": [round(v, 6) for v in r["rph_decomp"]],
                         "rph_orig": [round(v, 6) for v in r["rph_orig"]],
                         "best_layers": r["best_layers"],
                         "best_layers_orig": 1 + int(np.argmax(r["rph_orig"]))})
    del x
    return rows


def study(Z, torch):
    """Rate-distortion sweep (Sec. V metrics) over the synthetic workloads:
    bit-rate, compression factor, PSNR, NRMSE, maximum error / bound,
    hitting rate and chosen m per relative bound, all metrics on the device."""
    import fieldgen as F
    import fieldgen.gpu as G
    fields = (("smooth3d_64", lambda: G.smooth3d((64, 64, 64), F.BASE_SEED + 0), (1,)),
              ("climate2d_1800x3600", lambda: G.climate2d((1800, 3600), F.BASE_SEED + 1), (1, 2)),
              ("cosmo3d_512_density", lambda: G.cosmo3d((512, 512, 512), F.BASE_SEED + 2), (1,)))
    rows = []
    for name, make, layer_set in fields:
        x = make()
        torch.cuda.synchronize()
        for nl in layer_set:
            for eb in (1e-2, 1e-3, 1e-4, 1e-5, 1e-6):
                print(f"[study] {name} layers {nl} eb_rel {eb:g}", file=sys.stderr, flush=True)
                row, xr, st = roundtrip(Z, torch, x, dict(layers=nl, m=0, eb_mode="rel", eb_rel=eb), steps=2)
                row.update(quality_row(Z, x, xr, st.eb_used, max_lag=1))
                row.update({"field": name, "layers": nl, "eb_rel": eb})
                rows.append(row)
                del xr
        del x
        torch.cuda.empty_cache()
    return {"rate_distortion": rows,
            "layer_study": layer_study(Z, torch, eb_rels=(1e-3, 1e-4, 1e-5, 1e-6))
            + layer_study(Z, torch, eb_rels=(1e-3, 1e-4, 1e-5), samples=(None, (64, 64, 64)), field="sines3d")}


def bench_batched(Z, torch, count=64, reps=5):
    """Batched form on the uneven 64-field mix (32 square 2D fields of side
    512..4096, 32 cubes of side 64..384, f32, per-field relative bounds
    1e-5..1e-3): autotuned persistent launch replayed as a HIP graph, against
    plain per-field sz_compress calls, with a byte-for-byte check per field."""
    import fieldgen as F
    import fieldgen.gpu as G
    specs = F.batch_fields(count)
    xs = [G.batch_field(s) for s in specs]
    kws = [dict(layers=1, m=8, eb_mode="rel", eb_rel=s["eb_rel"]) for s in specs]
    total = sum(x.numel() * x.element_size() for x in xs)
    ctx = Z.context(0)
    st = torch.cuda.current_stream().cuda_stream
    params = [Z.make_params(tuple(x.shape), "float32", **kw) for x, kw in zip(xs, kws)]
    caps = [Z.sz_compress_bound(p) for p in params]
    outs = [torch.empty(c, dtype=torch.uint8, device="cuda") for c in caps]
    sizes = [0] * len(xs)

    def plain():
        for i in range(len(xs)):
            rc, sizes[i], _ = Z.sz_compress(ctx, params[i], xs[i].data_ptr(), outs[i].data_ptr(), caps[i], st)
            if rc:
                raise Z.SzError(rc, "sz_compress")

    plain()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plain()
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / reps

    B = Z.Batch([x.shape for x in xs], "float32", kws, schedule=-1)
    t0 = time.perf_counter()
    B.compress_async(xs)  # autotunes, then captures the graph
    torch.cuda.synchronize()
    t_tune = time.perf_counter() - t0
    B.compress_async(xs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        B.compress_async(xs)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / reps
    bsz = B.sizes.cpu().tolist()
    bst = B.status.cpu().tolist()
    exact = all(s == 0 for s in bst) and all(
        bsz[i] == sizes[i] and torch.equal(B.outs[i][: sizes[i]], outs[i][: sizes[i]]) for i in range(len(xs)))
    sched, tiles, threads, ms = B.info()
    # on-device distortion of every field's container, decompressed by the plain path
    worst_ratio, min_psnr = 0.0, float("inf")
    for i, x in enumerate(xs):
        xr = Z.decompress(B.outs[i][: bsz[i]]).view(x.shape)
        q = Z.quality(x, xr)
        worst_ratio = max(worst_ratio, q["max_abs_err"] / (kws[i]["eb_rel"] * q["value_range"]))
        min_psnr = min(min_psnr, q["psnr"])
        del xr
    B.close()
    return {"fields": len(xs), "input_bytes": int(total), "plain_ms": round(t_plain * 1e3, 3),
            "batched_ms": round(t_batch * 1e3, 3), "plain_GBps": round(total / t_plain / 1e9, 3),
            "batched_GBps": round(total / t_batch / 1e9, 3), "speedup": round(t_plain / t_batch, 3),
            "bit_exact_vs_plain": bool(exact), "schedule": sched, "sweep_tiles": tiles,
            "threads_per_sweep_wg": threads, "tune_ms": [round(v, 3) for v in ms],
            "tune_wall_s": round(t_tune, 3), "graph": True,
            "quality": {"min_psnr_db": round(min_psnr, 3), "max_err_over_eb": round(worst_ratio, 6)}}


def bench_served(Z, torch, rates=(10, 20, 50, 100, 200, 500), durations=(3.0, 2.0, 1.0, 0.8, 0.6, 0.4), slots=8,
                 budget=6 << 30):
    """Served form: Poisson arrivals of compress/decompress requests (sizes
    lognormal, median 32 MB, clipped to [1 MB, 2 GB], 80/20 f32/f64, 1-3D,
    relative bounds 1e-6..1e-3) at each rate, through the request server with
    `slots` concurrent slots and an HBM budget that binds (a request's input,
    output capacity and workspace count against it; the largest request
    needs about 5 GB), against plain per-call sz_compress / sz_decompress on
    one host thread in arrival order (a sequential FIFO).  Decompress
    requests carry the host copy of their container header, as a client that
    made the container has it.  Latency = completion - arrival."""
    import fieldgen as F
    import fieldgen.gpu as G
    out = {"slots": slots, "hbm_budget_bytes": int(budget), "rates": []}
    ctx = Z.context(0)
    for k, (rate, duration) in enumerate(zip(rates, durations)):
        reqs = F.request_stream(rate, duration, seed=F.BASE_SEED + 40 + k)
        print(f"[bench] served: rate {rate}/s, {len(reqs)} requests", file=sys.stderr, flush=True)
        data = []
        for r in reqs:
            data.append(G.request_field(r))
            torch.cuda.synchronize()
        kws = [dict(layers=1, m=8, eb_mode="rel", eb_rel=r["eb_rel"]) for r in reqs]
        comps, hdrs = {}, {}
        for i, r in enumerate(reqs):
            if r["op"] == "decompress":
                comps[i] = Z.compress(data[i], **kws[i])[0].clone()
                hdrs[i] = comps[i][:HEADER].cpu().numpy().tobytes()
        torch.cuda.synchronize()
        print("[bench] served: inputs and containers made", file=sys.stderr, flush=True)
        nbytes = sum(x.numel() * x.element_size() for x in data)
        row = {"rate": rate, "duration_s": duration, "requests": len(reqs), "bytes": int(nbytes),
               "largest_request_bytes": int(max(x.numel() * x.element_size() for x in data))}
        outs = []
        for i, (r, x) in enumerate(zip(reqs, data)):
            if r["op"] == "compress":
                cap = Z.sz_compress_bound(Z.make_params(tuple(x.shape), x.dtype, **kws[i]))
                outs.append(torch.empty(cap, dtype=torch.uint8, device="cuda"))
            else:
                outs.append(torch.empty_like(x))
        for mode in ("served", "plain"):
            t0 = time.perf_counter()
            if mode == "served":
                srv = Z.Server(budget, slots)
                ids = []
                for i, r in enumerate(reqs):
                    dt = t0 + r["t"] - time.perf_counter()
                    if dt > 0:
                        time.sleep(dt)
                    if r["op"] == "compress":
                        ids.append(srv.submit_compress(data[i], outs[i], **kws[i]))
                    else:
                        ids.append(srv.submit_decompress(comps[i], outs[i], header=hdrs[i]))
                res = []
                for n_done, i in enumerate(ids):
                    res.append(srv.wait(i, timeout_ms=120000))
                    if n_done % 50 == 49:
                        print(f"[bench] served: {n_done + 1} done", file=sys.stderr, flush=True)
                stats = srv.stats()
                srv.close()
                lat = np.array([x["t_done"] - x["t_submit"] for x in res]) * 1e3
                wait = np.array([x["t_admit"] - x["t_submit"] for x in res]) * 1e3
                span = max(x["t_done"] for x in res) - min(x["t_submit"] for x in res)
                errs = sum(1 for x in res if x["status"])
                codes = sorted({int(x["status"]) for x in res if x["status"]})
            else:
                # plain calls, one at a time in arrival order, each waiting for
                # its arrival; latency from arrival to the call's return
                stream = torch.cuda.current_stream().cuda_stream
                lat, errs, codes = [], 0, set()
                for i, r in enumerate(reqs):
                    dt = t0 + r["t"] - time.perf_counter()
                    if dt > 0:
                        time.sleep(dt)
                    if r["op"] == "compress":
                        p = Z.make_params(tuple(data[i].shape), data[i].dtype, **kws[i])
                        rc, _, _ = Z.sz_compress(ctx, p, data[i].data_ptr(), outs[i].data_ptr(), outs[i].numel(),
                                                 stream)
                    else:
                        rc = Z.sz_decompress(ctx, comps[i].data_ptr(), comps[i].numel(), outs[i].data_ptr(),
                                             outs[i].numel() * outs[i].element_size(), stream)
                    errs += rc != 0
                    if rc:
                        codes.add(int(rc))
                    lat.append(time.perf_counter() - (t0 + r["t"]))
                lat = np.array(lat) * 1e3
                span = time.perf_counter() - (t0 + reqs[0]["t"])
            print(f"[bench] served: {mode} finished", file=sys.stderr, flush=True)
            row[mode] = {"p50_ms": round(float(np.percentile(lat, 50)), 3),
                         "p99_ms": round(float(np.percentile(lat, 99)), 3),
                         "GBps": round(nbytes / span / 1e9, 3), "errors": int(errs),
                         "error_codes": sorted(codes)}
            if mode == "served":
                row[mode].update({"admission_wait_p50_ms": round(float(np.percentile(wait, 50)), 3),
                                  "admission_wait_p99_ms": round(float(np.percentile(wait, 99)), 3),
                                  "max_in_flight": stats["max_in_flight"],
                                  "peak_footprint_bytes": stats["pool_peak_bytes"]})
                # on-device distortion of every compress result and every
                # decompress result against its original field
                worst, min_psnr = 0.0, float("inf")
                for i, r in enumerate(reqs):
                    if res[i]["status"]:
                        continue
                    if r["op"] == "compress":
                        xr = Z.decompress(outs[i][: res[i]["out_size"]]).view(data[i].shape)
                    else:
                        xr = outs[i]
                    q = Z.quality(data[i], xr)
                    worst = max(worst, q["max_abs_err"] / (kws[i]["eb_rel"] * q["value_range"]))
                    min_psnr = min(min_psnr, q["psnr"])
                    del xr
                row[mode]["quality"] = {"min_psnr_db": round(min_psnr, 3), "max_err_over_eb": round(worst, 6)}
        out["rates"].append(row)
        del outs, data, comps
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-planes", type=int, default=32)
    ap.add_argument("--cpu-workers", type=int, default=16,
                    help="processes of the all-cores oracle figure (0 skips it)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the velocity / f64 cosmology runs and the layer study")
    ap.add_argument("--study", action="store_true",
                    help="only run the rate-distortion sweep and the best-layer study")
    ap.add_argument("--copy-ref", action="store_true",
                    help="only run a plain 512 MiB device copy (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}); "
              "the single-GPU kernel is the unit a multi-GPU run would shard.", file=sys.stderr)
        sys.exit(2)

    import torch
    import fieldgen as F
    import fieldgen.gpu as G
    import paper_1706_03791_amd as Z

    if args.copy_ref:
        a = torch.ones(1 << 27, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_ref_bytes": a.numel() * 4, "launches": 3}), flush=True)
        return

    if args.study:
        print(json.dumps(study(Z, torch)), flush=True)
        return

    n = args.size
    kw = dict(layers=1, m=8, eb_mode="rel", eb_rel=1e-4)
    print(f"[bench] generating {n}^3 field", file=sys.stderr, flush=True)
    xd = G.cosmo3d((n, n, n), F.BASE_SEED + 2)
    torch.cuda.synchronize()
    S = xd.numel() * xd.element_size()
    p = Z.make_params(tuple(xd.shape), "float32", **kw)
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
    # Inside the timed steps only the two sweeps (one of which is the
    # dominant kernel) record events: every timed stage adds two event
    # records to the stream.  The other stages' times come from untimed steps
    # with every stage timed.
    Z.sz_ctx_profile(ctx, True, stages=SWEEP_STAGES)
    torch.cuda.synchronize()
    tc, td = [], []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        a, b, size, st = step()
        tc.append(a)
        td.append(b)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    prof_timed = Z.sz_ctx_profile_read(ctx)
    print(f"[bench] timed {args.steps} steps in {t_total:.3f} s", file=sys.stderr, flush=True)
    Z.sz_ctx_profile(ctx, True)
    for _ in range(BREAKDOWN_STEPS):
        step()
    torch.cuda.synchronize()
    prof = merge_profiles(Z.sz_ctx_profile_read(ctx), prof_timed)
    Z.sz_ctx_profile(ctx, False)

    # correctness guard on the last step: the bound holds everywhere
    err = (out.double() - xd.double()).abs().max().item()
    assert err < st.eb_used, (err, st.eb_used)

    quality = quality_row(Z, xd, out, st.eb_used, max_lag=4)

    Cb = size
    t_c, t_d = float(np.median(tc)), float(np.median(td))
    value = 2 * S / (t_c + t_d) / 1e9
    # a plain device copy of the field for scale (reads S, writes S)
    cp = torch.empty_like(xd)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    cp.copy_(xd)
    e0.record()
    for _ in range(10):
        cp.copy_(xd)
    e1.record()
    torch.cuda.synchronize()
    copy_gbps = 2 * S / (e0.elapsed_time(e1) / 10 / 1e3) / 1e9
    del cp
    alg_bytes = (2 * S + Cb) + (Cb + S)
    hbm_frac = alg_bytes / (t_c + t_d) / 1e9 / HBM_PEAK_GBPS

    # dominant kernel stage and its algorithmic bytes per launch
    per_call = {k: (ms / calls if calls else 0.0) for k, (ms, calls) in prof.items()}
    npts = S // 4
    roof = stage_roofline(per_call, S, Cb, npts, 1)
    dom, dom_ms = roof["kernel"], roof["launch_ms"]
    traffic = load_traffic(dom, f"cosmo{n}", roof["algorithmic_bytes_per_launch"])
    roof["traffic"] = traffic
    if traffic:
        # counter-measured HBM bytes over the same launch time, beside the
        # algorithmic figure of `achieved`
        roof["traffic_GBps"] = round(traffic / (dom_ms / 1e3) / 1e9, 2)
        roof["traffic_frac"] = round(traffic / (dom_ms / 1e3) / 1e9 / HBM_PEAK_GBPS, 4)

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
                               f"m=8, eb_rel=1e-4, compress+decompress", "n_points": int(xd.numel()),
                   "field_bytes": int(S), "generator": "fieldgen.gpu.cosmo3d (torch, seed 20170614)"},
        "compress_GBps": round(S / t_c / 1e9, 3),
        "decompress_GBps": round(S / t_d / 1e9, 3),
        "hbm_frac": round(hbm_frac, 4),
        "compression_factor": round(S / Cb, 3),
        "bit_rate": round(8.0 * Cb / xd.numel(), 4),
        "m_used": int(st.m_used),
        "m_suggested": int(st.m_suggested),
        "device_copy_GBps": round(copy_gbps, 1),
        "timing": "median per-step compress and decompress times over the timed steps; stage_ms of the sweeps from HIP events in the timed steps, of the other stages from 3 untimed steps with every stage timed",
        "hit_rate": st.hit_rate,
        "n_unpred": int(st.n_unpred),
        "quality": quality,
        "stage_ms": {k: round(v, 4) for k, v in per_call.items()},
        "roofline": roof,
    }
    x_host = xd.cpu().numpy() if not args.no_cpu_baseline else None
    x_slab = x_host[: args.cpu_planes] if x_host is not None else None
    del xd, out, comp
    torch.cuda.empty_cache()
    if not args.no_extras:
        res["cosmology_extras"] = bench_cosmo_extras(Z, torch, n)
        print("[bench] layer study", file=sys.stderr, flush=True)
        res["layer_study"] = layer_study(Z, torch)
    if not args.no_batched:
        print("[bench] batched form", file=sys.stderr, flush=True)
        res["batched"] = bench_batched(Z, torch)
    if not args.no_served:
        print("[bench] served form", file=sys.stderr, flush=True)
        res["served"] = bench_served(Z, torch)
        res["p99_latency_served_ms"] = res["served"]["rates"][-1]["served"]["p99_ms"]
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(x_slab, args.cpu_planes, kw)
        if args.cpu_workers > 0:
            print("[bench] cpu baseline, all cores (oracle on slabs)", file=sys.stderr, flush=True)
            res["cpu_baseline_all_cores"] = cpu_all_cores(x_host, args.cpu_planes, kw, args.cpu_workers)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
