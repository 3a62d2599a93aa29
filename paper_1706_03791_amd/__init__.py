"""MI355X (gfx950) error-bounded lossy compressor of arXiv 1706.03791 (SZ-1.4).

Thin ctypes binding of the C ABI in ``include/szhip.h``: the functions named
``sz_*`` mirror the C entry points one to one (argument marshalling only);
``compress`` / ``decompress`` are conveniences over torch tensors on the GPU.
Every step of the method runs in the HIP kernels of ``libszhip.so``; there is
no CPU fallback -- importing the binding without the built library raises.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libszhip.so")

SZ_OK, SZ_EINVAL, SZ_ECAPACITY, SZ_ECORRUPT, SZ_ENONFINITE, SZ_ENOMEM, SZ_EHIP, SZ_ESTALL = 0, -1, -2, -3, -4, -5, -6, -7
SZ_ETIMEDOUT = -8
SZ_ESCRATCH = -9
SZ_NOALLOC_SCRATCH_BYTES = 256 << 20
SZ_REQ_COMPRESS, SZ_REQ_DECOMPRESS = 0, 1
SZ_F32, SZ_F64 = 0, 1
SZ_EB_ABS, SZ_EB_REL, SZ_EB_ABS_AND_REL = 0, 1, 2
HEADER_BYTES = 192

EXPORTS = ("sz_ctx_create", "sz_ctx_destroy", "sz_compress_bound", "sz_compress", "sz_compress_async",
           "sz_compress_async_noalloc",
           "sz_inspect", "sz_decompress", "sz_quantize", "sz_strerror", "sz_ctx_profile",
           "sz_ctx_profile_read", "sz_ctx_debug_sweep", "sz_batch_create", "sz_batch_compress", "sz_batch_info",
           "sz_batch_destroy", "sz_server_create", "sz_server_submit", "sz_server_wait", "sz_server_stats",
           "sz_server_destroy", "sz_quality", "sz_layer_survey")
STAGES = ("range", "sweep_compress", "codebook", "encode", "dectab", "decode", "unpred", "sweep_decompress",
          "hist")


class SzParams(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("dtype", C.c_uint32), ("ndim", C.c_uint32), ("dims", C.c_uint64 * 3),
                ("block", C.c_uint64 * 3), ("layers", C.c_uint32), ("quant_bits", C.c_uint32),
                ("eb_mode", C.c_uint32), ("chunk", C.c_uint32), ("eb_abs", C.c_double),
                ("eb_rel", C.c_double), ("theta", C.c_double), ("unpred_coding", C.c_uint32),
                ("reserved", C.c_uint32)]


class SzStats(C.Structure):
    _fields_ = [("n_points", C.c_uint64), ("n_unpred", C.c_uint64), ("huff_bits", C.c_uint64),
                ("tail_bits", C.c_uint64), ("compressed_bytes", C.c_uint64), ("ebT_bits", C.c_uint64),
                ("eb_used", C.c_double), ("hit_rate", C.c_double), ("value_min", C.c_double),
                ("value_max", C.c_double), ("m_used", C.c_uint32), ("m_suggested", C.c_uint32),
                ("raw_fallback", C.c_uint32), ("n_used_syms", C.c_uint32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SzRequest(C.Structure):
    _fields_ = [("op", C.c_uint32), ("reserved", C.c_uint32), ("params", SzParams), ("d_in", C.c_void_p),
                ("in_bytes", C.c_size_t), ("h_header", C.c_void_p), ("d_out", C.c_void_p), ("out_cap", C.c_size_t)]


class SzResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("slot", C.c_uint32), ("out_size", C.c_uint64),
                ("workspace_bytes", C.c_uint64), ("t_submit", C.c_double), ("t_admit", C.c_double),
                ("t_done", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SzServerStats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("admitted", C.c_uint64), ("completed", C.c_uint64),
                ("in_flight", C.c_uint32), ("max_in_flight", C.c_uint32), ("pool_bytes", C.c_uint64),
                ("pool_peak_bytes", C.c_uint64), ("clock_s", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SzQuality(C.Structure):
    _fields_ = [("n", C.c_uint64), ("value_min", C.c_double), ("value_max", C.c_double),
                ("value_range", C.c_double), ("max_abs_err", C.c_double), ("mean_err", C.c_double),
                ("rmse", C.c_double), ("nrmse", C.c_double), ("psnr", C.c_double), ("pearson", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SzError(RuntimeError):
    def __init__(self, code: int, where: str = ""):
        super().__init__(f"{where}: {strerror(code)} ({code})")
        self.code = code


_lib = None
_lock = threading.Lock()


def lib():
    """The loaded HIP library (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"HIP library missing: {LIB_PATH} (run paper_1706_03791_amd.build.build())")
            L = C.CDLL(LIB_PATH)
            vp, P = C.c_void_p, C.POINTER
            L.sz_ctx_create.argtypes = [P(vp), C.c_int]
            L.sz_ctx_destroy.argtypes = [vp]
            L.sz_ctx_destroy.restype = None
            L.sz_compress_bound.argtypes = [P(SzParams)]
            L.sz_compress_bound.restype = C.c_size_t
            L.sz_compress.argtypes = [vp, P(SzParams), vp, vp, C.c_size_t, P(C.c_size_t), P(SzStats), vp]
            L.sz_compress_async.argtypes = [vp, P(SzParams), vp, vp, C.c_size_t, vp, vp, vp]
            L.sz_compress_async_noalloc.argtypes = [vp, P(SzParams), vp, vp, C.c_size_t, vp, vp, vp]
            L.sz_inspect.argtypes = [vp, C.c_size_t, P(SzParams), P(SzStats)]
            L.sz_decompress.argtypes = [vp, vp, C.c_size_t, vp, C.c_size_t, vp]
            L.sz_quantize.argtypes = [vp, P(SzParams), vp, vp, vp, P(SzStats), vp]
            L.sz_strerror.argtypes = [C.c_int]
            L.sz_strerror.restype = C.c_char_p
            L.sz_ctx_profile.argtypes = [vp, C.c_int]
            L.sz_ctx_profile_read.argtypes = [vp, vp, vp, C.c_int]
            L.sz_ctx_debug_sweep.argtypes = [vp, C.c_int, C.c_int]
            L.sz_batch_create.argtypes = [vp, C.c_uint32, P(SzParams), C.c_int, P(vp)]
            L.sz_batch_compress.argtypes = [vp, vp, vp, vp, vp, vp, C.c_int, vp]
            L.sz_batch_info.argtypes = [vp, P(C.c_int), P(C.c_uint32), P(C.c_int), vp, C.c_int]
            L.sz_batch_destroy.argtypes = [vp]
            L.sz_batch_destroy.restype = None
            L.sz_server_create.argtypes = [C.c_int, C.c_size_t, C.c_uint32, P(vp)]
            L.sz_server_submit.argtypes = [vp, P(SzRequest), P(C.c_uint64)]
            L.sz_server_wait.argtypes = [vp, C.c_uint64, P(SzResult), C.c_int]
            L.sz_server_stats.argtypes = [vp, P(SzServerStats)]
            L.sz_server_destroy.argtypes = [vp]
            L.sz_server_destroy.restype = None
            L.sz_quality.argtypes = [vp, C.c_uint32, C.c_uint64, vp, vp, C.c_uint32, vp, P(SzQuality), vp]
            L.sz_layer_survey.argtypes = [vp, P(SzParams), vp, vp, vp, vp, P(C.c_uint32), vp]
            _lib = L
        return _lib


def sz_strerror(code: int) -> str:
    return lib().sz_strerror(int(code)).decode()


def strerror(code: int) -> str:
    try:
        return sz_strerror(code)
    except RuntimeError:
        return f"error {code}"


# ------------------------------------------------------------ C ABI mirror
def sz_ctx_create(device: int = 0) -> int:
    h = C.c_void_p()
    rc = lib().sz_ctx_create(C.byref(h), int(device))
    if rc:
        raise SzError(rc, "sz_ctx_create")
    return h.value


def sz_ctx_destroy(ctx: int) -> None:
    lib().sz_ctx_destroy(C.c_void_p(ctx))


def sz_compress_bound(p: SzParams) -> int:
    return lib().sz_compress_bound(C.byref(p))


def sz_compress(ctx, p: SzParams, d_in: int, d_out: int, cap: int, stream: int = 0):
    """Returns (rc, out_size, stats)."""
    size = C.c_size_t(0)
    st = SzStats()
    rc = lib().sz_compress(C.c_void_p(ctx), C.byref(p), C.c_void_p(d_in), C.c_void_p(d_out), cap,
                           C.byref(size), C.byref(st), C.c_void_p(stream))
    return rc, size.value, st


def sz_compress_async(ctx, p: SzParams, d_in: int, d_out: int, cap: int, d_out_size: int, d_status: int,
                      stream: int = 0) -> int:
    return lib().sz_compress_async(C.c_void_p(ctx), C.byref(p), C.c_void_p(d_in), C.c_void_p(d_out), cap,
                                   C.c_void_p(d_out_size), C.c_void_p(d_status), C.c_void_p(stream))


def sz_compress_async_noalloc(ctx, p: SzParams, d_in: int, d_out: int, cap: int, d_out_size: int,
                              d_status: int, stream: int = 0) -> int:
    return lib().sz_compress_async_noalloc(C.c_void_p(ctx), C.byref(p), C.c_void_p(d_in), C.c_void_p(d_out), cap,
                                           C.c_void_p(d_out_size), C.c_void_p(d_status), C.c_void_p(stream))


def sz_inspect(header: bytes):
    """Returns (rc, params, stats) of a container header held in host memory."""
    buf = (C.c_uint8 * len(header)).from_buffer_copy(header)
    p, s = SzParams(), SzStats()
    rc = lib().sz_inspect(buf, len(header), C.byref(p), C.byref(s))
    return rc, p, s


def sz_decompress(ctx, d_comp: int, comp_size: int, d_out: int, cap: int, stream: int = 0) -> int:
    return lib().sz_decompress(C.c_void_p(ctx), C.c_void_p(d_comp), comp_size, C.c_void_p(d_out), cap,
                               C.c_void_p(stream))


def sz_quantize(ctx, p: SzParams, d_in: int, d_codes: int, d_xprime: int = 0, stream: int = 0):
    st = SzStats()
    rc = lib().sz_quantize(C.c_void_p(ctx), C.byref(p), C.c_void_p(d_in), C.c_void_p(d_codes),
                           C.c_void_p(d_xprime or None), C.byref(st), C.c_void_p(stream))
    return rc, st


def sz_ctx_profile(ctx, enable: bool = True, stages=None) -> int:
    """Per-stage event timing: off, every stage, or only the named stages."""
    value = int(enable)
    if enable and stages is not None:
        value = 0x10000 | sum(1 << STAGES.index(name) for name in stages)
    return lib().sz_ctx_profile(C.c_void_p(ctx), value)


def sz_ctx_debug_sweep(ctx, schedule: int, claim_order: int) -> int:
    return lib().sz_ctx_debug_sweep(C.c_void_p(ctx), int(schedule), int(claim_order))


def sz_ctx_profile_read(ctx):
    """Accumulated per-stage milliseconds and call counts as a dict."""
    ms = (C.c_double * 16)()
    calls = (C.c_uint64 * 16)()
    n = lib().sz_ctx_profile_read(C.c_void_p(ctx), ms, calls, 16)
    return {STAGES[i]: (ms[i], calls[i]) for i in range(min(n, len(STAGES)))}


def sz_batch_create(ctx, params, schedule: int = -1) -> int:
    """Plan a batch over a list of SzParams; returns the batch handle."""
    arr = (SzParams * len(params))(*params)
    h = C.c_void_p()
    rc = lib().sz_batch_create(C.c_void_p(ctx), len(params), arr, int(schedule), C.byref(h))
    if rc:
        raise SzError(rc, "sz_batch_create")
    return h.value


def sz_batch_compress(batch, d_in, d_out, caps, d_sizes: int, d_status: int, use_graph: bool = True,
                      stream: int = 0) -> int:
    n = len(d_in)
    ins = (C.c_void_p * n)(*d_in)
    outs = (C.c_void_p * n)(*d_out)
    cp = (C.c_size_t * n)(*caps)
    return lib().sz_batch_compress(C.c_void_p(batch), ins, outs, cp, C.c_void_p(d_sizes), C.c_void_p(d_status),
                                   int(bool(use_graph)), C.c_void_p(stream))


def sz_batch_info(batch):
    """(schedule, sweep tiles, threads per sweep workgroup, tuned ms per candidate)."""
    sched, tiles, thr = C.c_int(0), C.c_uint32(0), C.c_int(0)
    ms = (C.c_double * 8)()
    n = lib().sz_batch_info(C.c_void_p(batch), C.byref(sched), C.byref(tiles), C.byref(thr), ms, 8)
    return sched.value, tiles.value, thr.value, [ms[i] for i in range(n)]


def sz_batch_destroy(batch) -> None:
    lib().sz_batch_destroy(C.c_void_p(batch))


def sz_server_create(device: int, hbm_budget: int, slots: int) -> int:
    h = C.c_void_p()
    rc = lib().sz_server_create(int(device), int(hbm_budget), int(slots), C.byref(h))
    if rc:
        raise SzError(rc, "sz_server_create")
    return h.value


def sz_server_submit(server, req: SzRequest):
    """Returns (rc, request id)."""
    i = C.c_uint64(0)
    rc = lib().sz_server_submit(C.c_void_p(server), C.byref(req), C.byref(i))
    return rc, i.value


def sz_server_wait(server, rid: int, timeout_ms: int = -1):
    """Returns (rc, SzResult)."""
    r = SzResult()
    rc = lib().sz_server_wait(C.c_void_p(server), C.c_uint64(rid), C.byref(r), int(timeout_ms))
    return rc, r


def sz_server_stats(server) -> dict:
    s = SzServerStats()
    rc = lib().sz_server_stats(C.c_void_p(server), C.byref(s))
    if rc:
        raise SzError(rc, "sz_server_stats")
    return s.as_dict()


def sz_server_destroy(server) -> None:
    lib().sz_server_destroy(C.c_void_p(server))


def sz_quality(ctx, dtype: int, n: int, d_orig: int, d_recon: int, max_lag: int = 0, stream: int = 0):
    """Returns (rc, metrics dict, autocorrelation list of max_lag values)."""
    q = SzQuality()
    ac = (C.c_double * max(1, max_lag))()
    rc = lib().sz_quality(C.c_void_p(ctx), int(dtype), int(n), C.c_void_p(d_orig), C.c_void_p(d_recon),
                          int(max_lag), ac if max_lag else None, C.byref(q), C.c_void_p(stream))
    return rc, q.as_dict(), [ac[i] for i in range(max_lag)]


def sz_layer_survey(ctx, p: SzParams, d_in: int, sample=None, stream: int = 0):
    """Returns (rc, rph_decomp[4], rph_orig[4], best_n)."""
    smp = None
    if sample is not None:
        smp = (C.c_uint64 * 3)(*[int(v) for v in sample] + [0] * (3 - len(sample)))
    dec = (C.c_double * 4)()
    org = (C.c_double * 4)()
    best = C.c_uint32(0)
    rc = lib().sz_layer_survey(C.c_void_p(ctx), C.byref(p), C.c_void_p(d_in), smp, dec, org, C.byref(best),
                               C.c_void_p(stream))
    return rc, list(dec), list(org), best.value


# ------------------------------------------------------- torch conveniences
_ctx = {}


def context(device: int = 0) -> int:
    with _lock:
        pass
    if device not in _ctx:
        _ctx[device] = sz_ctx_create(device)
    return _ctx[device]


def make_params(shape, dtype="float32", layers=1, m=8, eb_mode="rel", eb_abs=0.0, eb_rel=0.0,
                block=None, chunk=0, theta=0.0, unpred_coding=0) -> SzParams:
    p = SzParams()
    p.struct_size = C.sizeof(SzParams)
    p.dtype = SZ_F32 if str(dtype).endswith("float32") else SZ_F64
    p.ndim = len(shape)
    for d, s in enumerate(shape):
        p.dims[d] = int(s)
    if block is not None:
        for d, b in enumerate(block):
            p.block[d] = int(b)
    p.layers = int(layers)
    p.quant_bits = int(m)
    p.eb_mode = {"abs": SZ_EB_ABS, "rel": SZ_EB_REL, "both": SZ_EB_ABS_AND_REL}[eb_mode] \
        if isinstance(eb_mode, str) else int(eb_mode)
    p.chunk = int(chunk)
    p.eb_abs = float(eb_abs)
    p.eb_rel = float(eb_rel)
    p.theta = float(theta)
    p.unpred_coding = int(unpred_coding)
    return p


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def compress(x, stream=None, out=None, **kw):
    """Compress a contiguous float32/float64 CUDA tensor.

    Returns (container uint8 tensor view, stats dict).  Keyword arguments are
    those of ``make_params`` (layers, m, eb_mode, eb_abs, eb_rel, block,
    chunk, theta).
    """
    import torch
    if not x.is_cuda or not x.is_contiguous():
        raise ValueError("x must be a contiguous device tensor")
    p = make_params(tuple(x.shape), x.dtype, **kw)
    cap = sz_compress_bound(p)
    if cap == 0:
        raise SzError(SZ_EINVAL, "compress")
    if out is None:
        out = torch.empty(cap, dtype=torch.uint8, device=x.device)
    rc, size, st = sz_compress(context(x.device.index or 0), p, x.data_ptr(), out.data_ptr(), out.numel(),
                               _stream(stream))
    if rc:
        raise SzError(rc, "sz_compress")
    return out[:size], st.as_dict()


def decompress(comp, stream=None, out=None):
    """Decompress a container held in a CUDA uint8 tensor; returns the field."""
    import torch
    hdr = bytes(comp[:HEADER_BYTES].cpu().numpy().tobytes())
    rc, p, _ = sz_inspect(hdr)
    if rc:
        raise SzError(rc, "sz_inspect")
    shape = tuple(int(p.dims[d]) for d in range(p.ndim))
    dt = torch.float32 if p.dtype == SZ_F32 else torch.float64
    if out is None:
        out = torch.empty(shape, dtype=dt, device=comp.device)
    rc = sz_decompress(context(comp.device.index or 0), comp.data_ptr(), comp.numel(), out.data_ptr(),
                       out.numel() * out.element_size(), _stream(stream))
    if rc:
        raise SzError(rc, "sz_decompress")
    return out


def quantize(x, m=8, stream=None, want_xprime=False, **kw):
    """Debug: codes (int32 tensor of the uint16 codes) of one sweep at fixed m."""
    import torch
    p = make_params(tuple(x.shape), x.dtype, m=m, **kw)
    codes = torch.empty(x.numel() + 8, dtype=torch.int16, device=x.device)
    xp = torch.empty_like(x) if want_xprime else None
    rc, st = sz_quantize(context(x.device.index or 0), p, x.data_ptr(), codes.data_ptr(),
                         xp.data_ptr() if xp is not None else 0, _stream(stream))
    if rc:
        raise SzError(rc, "sz_quantize")
    c = codes[: x.numel()].view(x.shape).to(torch.int32) & 0xFFFF
    return (c, xp, st.as_dict()) if want_xprime else (c, st.as_dict())


class Batch:
    """Batched compression of a fixed list of field shapes (torch tensors).

    ``kws`` is one keyword dict per field (those of ``make_params``); fields
    must share one dtype.  ``compress(xs)`` returns the containers as uint8
    tensor views, byte-identical to ``compress(x, **kw)`` field by field.
    """

    def __init__(self, shapes, dtype, kws, schedule=-1, device=0):
        import torch
        self.params = [make_params(tuple(s), dtype, **kw) for s, kw in zip(shapes, kws)]
        self.caps = [sz_compress_bound(p) for p in self.params]
        self.device = device
        self.handle = sz_batch_create(context(device), self.params, schedule)
        self.outs = [torch.empty(c, dtype=torch.uint8, device=f"cuda:{device}") for c in self.caps]
        self.sizes = torch.zeros(len(shapes), dtype=torch.int64, device=f"cuda:{device}")
        self.status = torch.zeros(len(shapes), dtype=torch.int32, device=f"cuda:{device}")

    def compress_async(self, xs, use_graph=True, stream=None):
        for x, p in zip(xs, self.params):
            if not x.is_cuda or not x.is_contiguous() or tuple(x.shape) != tuple(p.dims[d] for d in range(p.ndim)):
                raise ValueError("inputs must be contiguous device tensors of the planned shapes")
        rc = sz_batch_compress(self.handle, [x.data_ptr() for x in xs], [o.data_ptr() for o in self.outs],
                               self.caps, self.sizes.data_ptr(), self.status.data_ptr(), use_graph, _stream(stream))
        if rc:
            raise SzError(rc, "sz_batch_compress")

    def compress(self, xs, use_graph=True, stream=None):
        self.compress_async(xs, use_graph, stream)
        st = self.status.cpu().tolist()
        sz = self.sizes.cpu().tolist()
        for i, s in enumerate(st):
            if s:
                raise SzError(s, f"sz_batch_compress field {i}")
        return [o[:n] for o, n in zip(self.outs, sz)]

    def info(self):
        return sz_batch_info(self.handle)

    def close(self):
        if self.handle:
            sz_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Request server with continuous batching over torch device tensors.

    ``submit_compress(x, out, **kw)`` / ``submit_decompress(comp, out)``
    queue a request and return its id; ``wait(id)`` returns the result dict
    (status, out_size, t_submit, t_admit, t_done on the server clock).  The
    tensors must stay alive until ``wait`` returns.
    """

    def __init__(self, hbm_budget: int, slots: int = 4, device: int = 0):
        self.handle = sz_server_create(device, hbm_budget, slots)
        self._keep = {}

    def submit_compress(self, x, out, **kw):
        r = SzRequest()
        r.op = SZ_REQ_COMPRESS
        r.params = make_params(tuple(x.shape), x.dtype, **kw)
        r.d_in = x.data_ptr()
        r.d_out = out.data_ptr()
        r.out_cap = out.numel() * out.element_size()
        rc, rid = sz_server_submit(self.handle, r)
        if rc:
            raise SzError(rc, "sz_server_submit")
        self._keep[rid] = (x, out)
        return rid

    def submit_decompress(self, comp, out, header: bytes = None):
        r = SzRequest()
        r.op = SZ_REQ_DECOMPRESS
        r.d_in = comp.data_ptr()
        r.in_bytes = comp.numel()
        hb = None
        if header is not None:
            hb = (C.c_uint8 * len(header)).from_buffer_copy(header)
            r.h_header = C.cast(hb, C.c_void_p).value
        r.d_out = out.data_ptr()
        r.out_cap = out.numel() * out.element_size()
        rc, rid = sz_server_submit(self.handle, r)
        if rc:
            raise SzError(rc, "sz_server_submit")
        self._keep[rid] = (comp, out, hb)
        return rid

    def wait(self, rid, timeout_ms=-1):
        rc, r = sz_server_wait(self.handle, rid, timeout_ms)
        if rc:
            raise SzError(rc, "sz_server_wait")
        self._keep.pop(rid, None)
        return r.as_dict()

    def stats(self):
        return sz_server_stats(self.handle)

    def close(self):
        if self.handle:
            sz_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def quality(x, xr, max_lag=0, stream=None):
    """Error metrics of a reconstruction xr of x (device tensors of one dtype)."""
    import torch
    if x.shape != xr.shape or x.dtype != xr.dtype or not (x.is_contiguous() and xr.is_contiguous()):
        raise ValueError("x and xr must be contiguous tensors of one shape and dtype")
    rc, q, ac = sz_quality(context(x.device.index or 0), SZ_F32 if x.dtype == torch.float32 else SZ_F64,
                           x.numel(), x.data_ptr(), xr.data_ptr(), max_lag, _stream(stream))
    if rc:
        raise SzError(rc, "sz_quality")
    if max_lag:
        q["autocorr"] = ac
    return q


def layer_survey(x, sample=None, stream=None, **kw):
    """R_PH of n = 1..4 layers from decompressed and original values; best n."""
    p = make_params(tuple(x.shape), x.dtype, **kw)
    rc, dec, org, best = sz_layer_survey(context(x.device.index or 0), p, x.data_ptr(), sample, _stream(stream))
    if rc:
        raise SzError(rc, "sz_layer_survey")
    return {"rph_decomp": dec, "rph_orig": org, "best_layers": best}
