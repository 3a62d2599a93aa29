"""TEST INFRASTRUCTURE ONLY: ctypes wrapper of the plain sequential CPU oracle.

The oracle (``szref.c``) is a slow, obviously-sequential C implementation of the
SZ-1.4 compressor of arXiv 1706.03791 (Sec. III-A prediction, Sec. IV-A
quantization and Huffman coding, Sec. IV-B adaptive interval count,
Algorithm 1).  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package; the product
library never loads it, and the two share no code.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libszref.so")
_SRC = [os.path.join(_HERE, f) for f in ("szref.c", "szref_traverse.inc", "szref.h")]
_lock = threading.Lock()
_lib = None

OK, EINVAL, ECAPACITY, ECORRUPT, ENONFINITE, ENOMEM = 0, -1, -2, -3, -4, -5


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C11, no FMA contraction, no fast-math)."""
    newest = max(os.path.getmtime(f) for f in _SRC)
    if not force and os.path.exists(_SO) and os.path.getmtime(_SO) >= newest:
        return _SO
    tmp = _SO + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp,
           os.path.join(_HERE, "szref.c"), "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


class Params(C.Structure):
    _fields_ = [("dtype", C.c_uint32), ("ndim", C.c_uint32),
                ("dims", C.c_uint64 * 3), ("block", C.c_uint64 * 3),
                ("layers", C.c_uint32), ("quant_bits", C.c_uint32),
                ("eb_mode", C.c_uint32), ("chunk", C.c_uint32),
                ("eb_abs", C.c_double), ("eb_rel", C.c_double), ("theta", C.c_double),
                ("unpred_coding", C.c_uint32), ("reserved", C.c_uint32)]


class Stats(C.Structure):
    _fields_ = [("n_points", C.c_uint64), ("n_unpred", C.c_uint64),
                ("huff_bits", C.c_uint64), ("tail_bits", C.c_uint64),
                ("compressed_bytes", C.c_uint64), ("ebT_bits", C.c_uint64),
                ("eb_used", C.c_double), ("hit_rate", C.c_double),
                ("value_min", C.c_double), ("value_max", C.c_double),
                ("m_used", C.c_uint32), ("m_suggested", C.c_uint32),
                ("raw_fallback", C.c_uint32), ("n_used_syms", C.c_uint32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class EB(C.Structure):
    _fields_ = [("eb", C.c_double), ("ebT", C.c_double), ("twoeb", C.c_double),
                ("inv2eb", C.c_double), ("ebT_bits", C.c_uint64),
                ("twoeb_bits", C.c_uint64), ("inv2eb_bits", C.c_uint64),
                ("vmin", C.c_double), ("vmax", C.c_double)]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            path = os.environ.get("SZREF_LIB")
            if not path:
                path = build()
            L = C.CDLL(path)
            vp, P = C.c_void_p, C.POINTER
            L.szref_resolve_eb.argtypes = [P(Params), vp, P(EB)]
            L.szref_coefficients.argtypes = [C.c_uint32, C.c_uint32, vp, vp, C.c_int]
            L.szref_predict_original.argtypes = [P(Params), vp, vp]
            L.szref_quantize.argtypes = [P(Params), vp, C.c_uint32, vp, vp, P(C.c_uint64)]
            L.szref_huffman_lengths.argtypes = [vp, C.c_uint32, vp]
            L.szref_compress_bound.argtypes = [P(Params)]
            L.szref_compress_bound.restype = C.c_size_t
            L.szref_compress.argtypes = [P(Params), vp, P(C.POINTER(C.c_uint8)), P(C.c_size_t), P(Stats)]
            L.szref_compress_debug.argtypes = [P(Params), vp, P(C.POINTER(C.c_uint8)),
                                               P(C.c_size_t), P(Stats), vp, vp]
            L.szref_decompress.argtypes = [vp, C.c_size_t, vp, C.c_size_t]
            L.szref_inspect.argtypes = [vp, C.c_size_t, P(Params), P(Stats)]
            L.szref_free.argtypes = [vp]
            _lib = L
        return _lib


class OracleError(RuntimeError):
    def __init__(self, code, what=""):
        super().__init__(f"oracle error {code} {what}")
        self.code = code


def make_params(shape, dtype=np.float32, layers=1, m=8, eb_mode="abs", eb_abs=0.0,
                eb_rel=0.0, block=None, chunk=0, theta=0.0, unpred_coding=0) -> Params:
    p = Params()
    p.dtype = 0 if np.dtype(dtype) == np.float32 else 1
    p.ndim = len(shape)
    for d, s in enumerate(shape):
        p.dims[d] = int(s)
    if block is not None:
        for d, b in enumerate(block):
            p.block[d] = int(b)
    p.layers = layers
    p.quant_bits = m
    p.eb_mode = {"abs": 0, "rel": 1, "both": 2}[eb_mode] if isinstance(eb_mode, str) else int(eb_mode)
    p.chunk = chunk
    p.eb_abs = eb_abs
    p.eb_rel = eb_rel
    p.theta = theta
    p.unpred_coding = unpred_coding
    return p


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def resolve_eb(data: np.ndarray, **kw) -> dict:
    data = np.ascontiguousarray(data)
    p = make_params(data.shape, data.dtype, **kw)
    e = EB()
    rc = lib().szref_resolve_eb(C.byref(p), _ptr(data), C.byref(e))
    if rc:
        raise OracleError(rc, "resolve_eb")
    return {k: getattr(e, k) for k, _ in EB._fields_}


def coefficients(ndim: int, n: int):
    coef = np.zeros(124, np.int64)
    koff = np.zeros(124 * ndim, np.int32)
    c = lib().szref_coefficients(ndim, n, _ptr(coef), _ptr(koff), 124)
    if c < 0:
        raise OracleError(c, "coefficients")
    return coef[:c].copy(), koff[: c * ndim].reshape(c, ndim).copy()


def predict_original(data: np.ndarray, layers=1, block=None) -> np.ndarray:
    data = np.ascontiguousarray(data)
    p = make_params(data.shape, data.dtype, layers=layers, block=block)
    out = np.empty_like(data)
    rc = lib().szref_predict_original(C.byref(p), _ptr(data), _ptr(out))
    if rc:
        raise OracleError(rc, "predict_original")
    return out


def quantize(data: np.ndarray, m=8, **kw):
    """One traversal at fixed m: (codes u16, recorded decompressed values, n_unpred)."""
    data = np.ascontiguousarray(data)
    p = make_params(data.shape, data.dtype, m=m, **kw)
    codes = np.empty(data.shape, np.uint16)
    xp = np.empty_like(data)
    nu = C.c_uint64(0)
    rc = lib().szref_quantize(C.byref(p), _ptr(data), m, _ptr(codes), _ptr(xp), C.byref(nu))
    if rc:
        raise OracleError(rc, "quantize")
    return codes, xp, nu.value


def huffman_lengths(freq) -> np.ndarray:
    f = np.ascontiguousarray(np.asarray(freq, np.uint64))
    out = np.zeros(len(f), np.uint8)
    rc = lib().szref_huffman_lengths(_ptr(f), len(f), _ptr(out))
    if rc < 0:
        raise OracleError(rc, "huffman_lengths")
    return out


def compress(data: np.ndarray, debug=False, **kw):
    """Full compressor.  Returns (container bytes, stats dict[, codes, xprime])."""
    data = np.ascontiguousarray(data)
    p = make_params(data.shape, data.dtype, **kw)
    out = C.POINTER(C.c_uint8)()
    size = C.c_size_t(0)
    st = Stats()
    L = lib()
    if debug:
        codes = np.empty(data.shape, np.uint16)
        xp = np.empty_like(data)
        rc = L.szref_compress_debug(C.byref(p), _ptr(data), C.byref(out), C.byref(size),
                                    C.byref(st), _ptr(codes), _ptr(xp))
    else:
        rc = L.szref_compress(C.byref(p), _ptr(data), C.byref(out), C.byref(size), C.byref(st))
    if rc:
        raise OracleError(rc, "compress")
    buf = bytes(C.string_at(out, size.value))
    L.szref_free(out)
    if debug:
        return buf, st.as_dict(), codes, xp
    return buf, st.as_dict()


def decompress(buf: bytes) -> np.ndarray:
    info = inspect(buf)
    shape = tuple(info["dims"])
    dt = np.float32 if info["dtype"] == 0 else np.float64
    out = np.empty(shape, dt)
    arr = np.frombuffer(buf, np.uint8)
    rc = lib().szref_decompress(_ptr(arr), len(buf), _ptr(out), out.nbytes)
    if rc:
        raise OracleError(rc, "decompress")
    return out


def decompress_raw(buf: bytes, cap: int) -> int:
    """Return code of a decompression into a scratch buffer of `cap` bytes."""
    arr = np.frombuffer(buf, np.uint8)
    out = np.empty(max(cap, 1), np.uint8)
    return lib().szref_decompress(_ptr(arr), len(buf), _ptr(out), cap)


def inspect(buf: bytes) -> dict:
    arr = np.frombuffer(buf, np.uint8)
    p, s = Params(), Stats()
    rc = lib().szref_inspect(_ptr(arr), len(buf), C.byref(p), C.byref(s))
    if rc:
        raise OracleError(rc, "inspect")
    d = s.as_dict()
    d.update(dtype=p.dtype, ndim=p.ndim, dims=[p.dims[i] for i in range(p.ndim)],
             block=[p.block[i] for i in range(p.ndim)], layers=p.layers,
             quant_bits=p.quant_bits, eb_mode=p.eb_mode, chunk=p.chunk,
             eb_abs=p.eb_abs, eb_rel=p.eb_rel, unpred_coding=p.unpred_coding)
    return d
