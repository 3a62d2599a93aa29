"""Parity of the HIP path with the CPU oracle (MI355X only).

Every case runs the full compressor and decompressor through the C ABI and
requires, bit for bit: the container bytes (header, codebook, chunk table,
Huffman bitstream, heads and tails of unpredictable values) equal to the
oracle's, and the decompressed field equal to the values the oracle's
compressor recorded for later predictions.
"""
import numpy as np
import pytest

import fieldgen as F

pytestmark = pytest.mark.gpu

SECTIONS = [("header", 0, 136), ("codebook", 136, 144), ("chunks", 144, 152), ("bitstream", 152, 160),
            ("heads", 160, 168), ("tails", 168, 176)]


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


def _u(a):
    return a.view(np.uint32 if a.dtype == np.float32 else np.uint64)


def _locate(got: bytes, ref: bytes) -> str:
    if len(got) < 192 or len(ref) < 192:
        return f"sizes {len(got)} vs {len(ref)}"
    g = np.frombuffer(got, np.uint8)
    r = np.frombuffer(ref, np.uint8)
    n = min(len(g), len(r))
    d = np.nonzero(g[:n] != r[:n])[0]
    if not len(d):
        return f"prefix equal, sizes {len(got)} vs {len(ref)}"
    first = int(d[0])
    offs = [int.from_bytes(ref[o:o + 8], "little") for o in range(136, 184, 8)]
    names = ["header", "codebook", "chunks", "bitstream", "heads", "tails"]
    starts = [0] + offs[:5]
    sec = "?"
    for nm, st in zip(names, starts):
        if first >= st:
            sec = nm
    return f"first differing byte {first} in section {sec}; {len(d)} bytes differ; sizes {len(got)} vs {len(ref)}"


def check(Z, oracle, x, **kw):
    ref, sref, codes_ref, xp_ref = oracle.compress(x, debug=True, **kw)
    comp, st = Z.compress(dev(x), **kw)
    got = comp.cpu().numpy().tobytes()
    if got != ref:
        c, _ = Z.quantize(dev(x), **dict(kw, m=sref["m_used"]))
        cg = c.cpu().numpy().astype(np.uint16)
        bad = np.argwhere(cg != codes_ref)
        raise AssertionError(_locate(got, ref) + f"; code mismatches {len(bad)} first {bad[:3].tolist()}")
    for k in ("n_unpred", "huff_bits", "tail_bits", "m_used", "m_suggested", "raw_fallback", "n_used_syms",
              "ebT_bits"):
        assert st[k] == sref[k], (k, st[k], sref[k])
    out = Z.decompress(comp).cpu().numpy()
    want = x if sref["raw_fallback"] else xp_ref
    assert np.array_equal(_u(out), _u(want))
    return sref


SHAPES = [
    (64, 64, 64), (19, 37, 45), (33, 70, 129), (1, 1, 700), (300, 1, 1), (17, 1, 300), (1, 300, 17),
    (90, 130), (600, 257), (1, 4000), (3000, 1), (10000,), (2048 * 5 + 7,), (1,), (100,),
]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("layers", [1, 2])
def test_shapes_f32(Z, oracle, shape, layers):
    rng = np.random.default_rng(len(shape) * 1000 + sum(shape))
    if len(shape) == 3 and min(shape) > 4:
        x = F.smooth3d(shape)
    else:
        x = np.cumsum(rng.normal(0, 1, int(np.prod(shape)))).reshape(shape).astype(np.float32)
    check(Z, oracle, x, layers=layers, m=8, eb_mode="rel", eb_rel=1e-4)


@pytest.mark.parametrize("layers", [1, 2, 3, 4])
@pytest.mark.parametrize("ndim", [1, 2, 3])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_layers_dtypes(Z, oracle, layers, ndim, dtype):
    shape = {1: (9000,), 2: (150, 170), 3: (24, 40, 50)}[ndim]
    x = (F.smooth3d((24, 40, 50)) if ndim == 3 else
         F.climate2d((150, 170)) if ndim == 2 else
         np.cumsum(np.random.default_rng(7).normal(0, 1, 9000)))
    x = np.ascontiguousarray(x).astype(dtype).reshape(shape)
    eb = 1e-5 if dtype == np.float32 else 1e-9
    check(Z, oracle, x, layers=layers, m=0, eb_mode="rel", eb_rel=eb)


@pytest.mark.parametrize("m", [1, 2, 5, 8, 9, 12, 16, 0])
def test_interval_counts(Z, oracle, m):
    x = F.climate2d((200, 300))
    check(Z, oracle, x, layers=1, m=m, eb_mode="rel", eb_rel=1e-5)


@pytest.mark.parametrize("mode,kw", [("abs", dict(eb_abs=0.05)), ("rel", dict(eb_rel=3e-4)),
                                     ("both", dict(eb_abs=0.01, eb_rel=1e-3)),
                                     ("both", dict(eb_abs=1.0, eb_rel=1e-5))])
def test_bound_modes(Z, oracle, mode, kw):
    x = F.smooth3d((30, 40, 50))
    check(Z, oracle, x, layers=1, m=8, eb_mode=mode, **kw)


@pytest.mark.parametrize("shape,block", [((40, 50, 60), (16, 20, 24)), ((300, 400), (100, 128)),
                                         ((50000,), (1000,)), ((35, 45, 33), (35, 10, 33)),
                                         ((20, 30, 40), (7, 30, 13)), ((700000,), (999,)),
                                         ((300001,), (4096,)), ((2000, 70), (1, 70))])
def test_blocks(Z, oracle, shape, block):
    x = (F.smooth3d(shape) if len(shape) == 3 else F.climate2d(shape) if len(shape) == 2 else
         np.cumsum(np.random.default_rng(3).normal(0, 1, shape[0])).astype(np.float32))
    check(Z, oracle, x, layers=1, m=8, eb_mode="rel", eb_rel=1e-4, block=block)
    check(Z, oracle, x, layers=2, m=0, eb_mode="rel", eb_rel=1e-4, block=block)


@pytest.mark.parametrize("chunk", [256, 512, 2048, 4096])
def test_chunk_sizes(Z, oracle, chunk):
    x = F.climate2d((123, 457))
    check(Z, oracle, x, layers=1, m=8, eb_mode="rel", eb_rel=1e-4, chunk=chunk)


@pytest.mark.parametrize("xorc", [0, 1], ids=["kept-bits", "xor"])
@pytest.mark.parametrize("chunk", [256, 512, 1024, 2048])
@pytest.mark.parametrize("dtype", [np.float32, np.float64], ids=["f32", "f64"])
def test_dense_unpredictable_encoder_forms(Z, oracle, dtype, chunk, xorc):
    """Fields with most values unpredictable (a random walk along x plus
    sparse noise, 16 bins): chunks of up to 1024 codes take the encoder form
    that keeps each lane's values in registers (f64 always, f32 when more
    than one value in 16 is unpredictable), longer chunks the form that loads
    them in every pass.  Both give the oracle's bytes (Sec. IV-B, Algorithm 1
    step storing the unpredictable value)."""
    rng = np.random.default_rng(11 + chunk)
    shape = (24, 30, 37)
    walk = np.cumsum(rng.normal(0, 1, shape), axis=2)
    x = (walk + rng.normal(0, 0.5, shape) * (rng.random(shape) < 0.3)).astype(dtype)
    s = check(Z, oracle, x, layers=1, m=4, eb_mode="rel", eb_rel=1e-3, chunk=chunk, unpred_coding=xorc)
    assert s["n_unpred"] * 16 > x.size
    assert s["n_unpred"] < x.size


def test_constant_field(Z, oracle):
    x = np.full((20, 30, 40), 3.25, np.float32)
    check(Z, oracle, x, layers=1, m=8, eb_mode="abs", eb_abs=1e-3)


def test_nonfinite_abs_mode(Z, oracle):
    x = F.smooth3d((20, 30, 40))
    x[3, 4, 5] = np.nan
    x[10, 0, 0] = np.inf
    x[0, 29, 39] = -np.inf
    check(Z, oracle, x, layers=1, m=8, eb_mode="abs", eb_abs=1e-3)


def test_nonfinite_rel_mode_rejected(Z):
    x = F.smooth3d((20, 30, 40))
    x[3, 4, 5] = np.nan
    with pytest.raises(Z.SzError) as e:
        Z.compress(dev(x), eb_mode="rel", eb_rel=1e-3)
    assert e.value.code == Z.SZ_ENONFINITE


def test_lossless_and_subnormals(Z, oracle):
    x = np.random.default_rng(2).normal(0, 1, (30, 40)).astype(np.float32)
    x[0, 0] = np.float32(1e-40)
    x[5, 5] = np.float32(-3e-42)
    check(Z, oracle, x, layers=1, m=8, eb_mode="abs", eb_abs=0.0)
    check(Z, oracle, x, layers=2, m=8, eb_mode="abs", eb_abs=1e-41)


def test_raw_fallback(Z, oracle):
    x = np.random.default_rng(4).normal(0, 1, 4096).astype(np.float32)
    s = check(Z, oracle, x, layers=1, m=8, eb_mode="abs", eb_abs=1e-30)
    assert s["raw_fallback"] == 1


def test_spiky_2d_full_size(Z, oracle):
    """Climate-like field at the ATM shape (Table III) with 1% spikes, both
    layer counts, the four relative bounds, adaptive m."""
    x = F.climate2d()
    for layers in (1, 2):
        for eb in (1e-3, 1e-4, 1e-5, 1e-6):
            check(Z, oracle, x, layers=layers, m=0, eb_mode="rel", eb_rel=eb)


def test_error_bound_on_gpu_output(Z):
    x = F.smooth3d((48, 64, 80))
    comp, st = Z.compress(dev(x), layers=1, m=8, eb_mode="rel", eb_rel=1e-5)
    out = Z.decompress(comp).cpu().numpy()
    assert np.max(np.abs(out.astype(np.float64) - x)) < st["eb_used"]


def test_corrupt_containers_rejected(Z):
    import torch
    x = F.smooth3d((24, 32, 40))
    comp, st = Z.compress(dev(x), layers=1, m=8, eb_mode="rel", eb_rel=1e-4)
    good = comp.cpu().numpy().copy()
    out = torch.empty(x.shape, dtype=torch.float32, device="cuda")
    ctx = Z.context(0)

    def run(buf):
        t = torch.from_numpy(buf).cuda()
        return Z.sz_decompress(ctx, t.data_ptr(), t.numel(), out.data_ptr(), out.numel() * 4,
                               torch.cuda.current_stream().cuda_stream)

    assert run(good) == 0
    assert run(good[:100].copy()) == Z.SZ_ECORRUPT
    assert run(good[:-8].copy()) == Z.SZ_ECORRUPT
    bad = good.copy()
    bad[0] ^= 1
    assert run(bad) == Z.SZ_ECORRUPT
    rng = np.random.default_rng(0)
    for _ in range(30):
        bad = good.copy()
        pos = int(rng.integers(192, len(bad)))
        bad[pos] ^= np.uint8(1 << int(rng.integers(0, 8)))
        assert run(bad) in (0, Z.SZ_ECORRUPT)
    assert run(good) == 0
    t = torch.from_numpy(good).cuda()
    assert Z.sz_decompress(ctx, t.data_ptr(), t.numel(), out.data_ptr(), 16,
                           torch.cuda.current_stream().cuda_stream) == Z.SZ_ECAPACITY


def test_capacity_error(Z):
    import torch
    x = F.smooth3d((24, 32, 40))
    p = Z.make_params(x.shape, "float32", layers=1, m=8, eb_mode="rel", eb_rel=1e-4)
    xi = dev(x)
    out = torch.empty(400, dtype=torch.uint8, device="cuda")
    rc, size, st = Z.sz_compress(Z.context(0), p, xi.data_ptr(), out.data_ptr(), 400,
                                 torch.cuda.current_stream().cuda_stream)
    assert rc == Z.SZ_ECAPACITY


XOR_CASES = [
    ("velocity 40x50x60 f32", lambda: __import__("fieldgen.gpu", fromlist=["x"]).velocity3d(
        (40, 50, 60), 5, device="cpu").numpy(), dict(layers=1, m=8, eb_mode="rel", eb_rel=1e-4)),
    ("velocity 33x70x129 f64", lambda: __import__("fieldgen.gpu", fromlist=["x"]).velocity3d(
        (33, 70, 129), 6, device="cpu").numpy().astype(np.float64), dict(layers=1, m=0, eb_mode="rel", eb_rel=1e-7)),
    ("climate 300x500 f32 2 layers", lambda: F.climate2d((300, 500)), dict(layers=2, m=0, eb_mode="rel", eb_rel=1e-6)),
    ("walk 50000 f32 chunk 256", lambda: np.cumsum(np.random.default_rng(8).normal(0, 20, 50000)).astype(np.float32),
     dict(layers=1, m=4, eb_mode="rel", eb_rel=1e-5, chunk=256)),
    ("walk 20001 f64 chunk 4096", lambda: np.cumsum(np.random.default_rng(9).normal(0, 20, 20001)),
     dict(layers=3, m=6, eb_mode="abs", eb_abs=1e-4, chunk=4096)),
    ("lossless 30x40 f32", lambda: np.random.default_rng(2).normal(0, 1, (30, 40)).astype(np.float32),
     dict(layers=1, m=8, eb_mode="abs", eb_abs=0.0)),
]


@pytest.mark.parametrize("case", range(len(XOR_CASES)), ids=[c[0] for c in XOR_CASES])
def test_xor_unpredictable_coding(Z, oracle, case):
    """Unpredictable values XOR-coded against the previous one of their
    chunk (container flag bit 1): bytes and decompressed bits equal the
    oracle's."""
    _, make, kw = XOR_CASES[case]
    x = np.ascontiguousarray(make())
    s = check(Z, oracle, x, unpred_coding=1, **kw)
    assert s["n_unpred"] > 0


def test_xor_coding_nonfinite(Z, oracle):
    x = F.smooth3d((20, 30, 40))
    x[3, 4, 5] = np.nan
    x[10, 0, 0] = np.inf
    x[0, 29, 39] = -np.inf
    x[7, 7, 7] = 1e30
    check(Z, oracle, x, layers=1, m=8, eb_mode="abs", eb_abs=1e-3, unpred_coding=1)
