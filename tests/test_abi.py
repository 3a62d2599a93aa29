"""The C-ABI library loads and exports what include/szhip.h declares (CPU).

Only host-side entry points are called here (no device work): the compress
bound, header inspection of an oracle-made container, error strings and
parameter validation.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def Z():
    import paper_1706_03791_amd as Z
    if not os.path.exists(Z.LIB_PATH):
        from paper_1706_03791_amd import build as B
        B.build()
    Z.lib()
    return Z


def declared_functions():
    with open(os.path.join(ROOT, "include", "szhip.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sz_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(Z):
    names = declared_functions()
    assert len(names) >= 9
    lib = C.CDLL(Z.LIB_PATH)
    for nm in names:
        assert hasattr(lib, nm), nm
    assert sorted(Z.EXPORTS) == names


def test_binding_names_mirror_the_abi(Z):
    for nm in declared_functions():
        assert callable(getattr(Z, nm)), nm


def test_strerror(Z):
    assert Z.strerror(0) == "ok"
    for code in (-1, -2, -3, -4, -5, -6, -7):
        assert Z.strerror(code) != "unknown error"


def test_compress_bound_and_validation(Z):
    p = Z.make_params((512, 512, 512), "float32", layers=1, m=8, eb_mode="rel", eb_rel=1e-4)
    assert Z.sz_compress_bound(p) == 192 + 512 ** 3 * 4
    p64 = Z.make_params((1800, 3600), "float64", layers=2, m=0, eb_mode="abs", eb_abs=1.0)
    assert Z.sz_compress_bound(p64) == 192 + 1800 * 3600 * 8
    for bad in (dict(layers=5), dict(layers=0), dict(m=17), dict(chunk=100), dict(chunk=8192),
                dict(eb_abs=-1.0, eb_mode="abs"), dict(eb_rel=float("nan"))):
        kw = dict(layers=1, m=8, eb_mode="rel", eb_rel=1e-4)
        kw.update(bad)
        assert Z.sz_compress_bound(Z.make_params((10, 10), "float32", **kw)) == 0, bad
    assert Z.sz_compress_bound(Z.make_params((0, 10), "float32", m=8)) == 0


def test_inspect_reads_oracle_header(Z, oracle):
    import fieldgen as F
    x = F.climate2d((120, 200))
    buf, st = oracle.compress(x, layers=2, m=0, eb_mode="rel", eb_rel=1e-4, chunk=512)
    rc, p, s = Z.sz_inspect(buf[:192])
    assert rc == 0
    assert (p.dtype, p.ndim, p.dims[0], p.dims[1], p.layers, p.quant_bits, p.chunk) == (0, 2, 120, 200, 2, 0, 512)
    assert p.eb_mode == Z.SZ_EB_REL and p.eb_rel == 1e-4
    assert s.n_unpred == st["n_unpred"] and s.huff_bits == st["huff_bits"]
    assert s.m_used == st["m_used"] and s.compressed_bytes == len(buf)
    rc, _, _ = Z.sz_inspect(b"\0" * 192)
    assert rc == Z.SZ_ECORRUPT
    rc, _, _ = Z.sz_inspect(buf[:100])
    assert rc == Z.SZ_ECORRUPT


def test_null_context_rejected(Z):
    p = Z.make_params((10, 10), "float32", m=8, eb_mode="abs", eb_abs=0.1)
    rc, _, _ = Z.sz_compress(0, p, 0, 0, 1000)
    assert rc == Z.SZ_EINVAL
    assert Z.sz_decompress(0, 0, 1000, 0, 1000) == Z.SZ_EINVAL


def test_header_declares_citations():
    with open(os.path.join(ROOT, "include", "szhip.h")) as f:
        text = f.read()
    for needle in ("Sec. III-A", "Sec. IV-A", "Sec. IV-B", "Algorithm 1", "Metric 1"):
        assert needle in text


def test_struct_size_checked(Z):
    p = Z.make_params((100, 100), "float32", layers=1, m=8, eb_mode="rel", eb_rel=1e-4)
    assert Z.sz_compress_bound(p) == 192 + 100 * 100 * 4
    p.struct_size = p.struct_size - 8  # a caller built against another layout
    assert Z.sz_compress_bound(p) == 0
    p.struct_size = 0
    assert Z.sz_compress_bound(p) == 0


def test_debug_sweep_argument_checks(Z):
    assert Z.sz_ctx_debug_sweep(0, 0, 0) == Z.SZ_EINVAL
