"""Pins of the CPU oracle to things other than itself (CPU only).

Each test checks the oracle against something the paper or mathematics fixes:
Table I, Theorem 1's exactness, the Lorenzo and finite-difference special
cases, hand-worked examples, brute force over tiny inputs, optimality of the
Huffman lengths by enumeration, and the error-bound invariant of Metric 1.
"""
import heapq
import itertools
import math
import struct
from fractions import Fraction

import numpy as np
import pytest

import fieldgen as F
from conftest import golden

# ----------------------------------------------------------- coefficients


def test_table1_coefficients(oracle):
    """Generic formula (Eq. predmodel) in 2D equals Table I row by row."""
    rows = golden("table1_2d_coefficients.txt")
    want = {}
    for key, vals in rows.items():
        for v in vals:
            want.setdefault(int(key), {})[(int(v[0]), int(v[1]))] = int(v[2])
    for n in range(1, 5):
        coef, koff = oracle.coefficients(2, n)
        got = {(int(k[0]), int(k[1])): int(c) for c, k in zip(coef, koff)}
        assert got == want[n], n
        assert len(got) == n * (n + 2)  # |S^n| = n(n+2) points (Sec. III-A)


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_coefficients_sum_to_one_and_count(oracle, d, n):
    coef, koff = oracle.coefficients(d, n)
    assert len(coef) == (n + 1) ** d - 1  # Algorithm 1: (n+1)^d - 1 coefficients
    assert int(coef.sum()) == 1  # a constant field is predicted exactly
    # lexicographic order, slowest dimension outermost
    keys = [tuple(k) for k in koff]
    assert keys == sorted(keys)


def test_3d_lorenzo_stencil(oracle):
    """n = 1 in 3D is the Lorenzo predictor: the 7 other corners of the unit
    cube with sign (-1)^(|k|+1)."""
    coef, koff = oracle.coefficients(3, 1)
    got = {tuple(int(x) for x in k): int(c) for c, k in zip(coef, koff)}
    want = {}
    for k in itertools.product((0, 1), repeat=3):
        if any(k):
            want[k] = 1 if sum(k) % 2 == 1 else -1
    assert got == want


def test_1d_finite_difference_extrapolation(oracle):
    """In 1D the n-layer model extrapolates the degree-(n-1) polynomial through
    the previous n points: coefficients (-1)^(k+1) C(n, k)."""
    assert list(oracle.coefficients(1, 1)[0]) == [1]
    assert list(oracle.coefficients(1, 2)[0]) == [2, -1]
    assert list(oracle.coefficients(1, 3)[0]) == [3, -3, 1]
    assert list(oracle.coefficients(1, 4)[0]) == [4, -6, 4, -1]


# ---------------------------------------------------- Theorem 1 exactness


def _poly_field(shape, monomials):
    grids = np.meshgrid(*[np.arange(s, dtype=np.float64) for s in shape], indexing="ij")
    f = np.zeros(shape, np.float64)
    for coef, exps in monomials:
        term = np.full(shape, float(coef))
        for g, e in zip(grids, exps):
            term = term * g ** e
        f += term
    return f


def _interior(shape, n):
    return tuple(slice(n, None) for _ in shape)


@pytest.mark.parametrize("case", [
    # (ndim, n, monomials [(coef, exps)], exact?)
    (2, 1, [(1, (3, 0)), (2, (0, 2)), (5, (0, 0))], True),   # g(i) + h(j)
    (2, 1, [(1, (1, 1))], False),                           # i*j: both exponents >= 1
    (2, 2, [(1, (5, 1)), (1, (1, 4)), (3, (3, 0))], True),  # each monomial has an exponent < 2
    (2, 2, [(1, (2, 2))], False),
    (2, 3, [(1, (2, 5)), (1, (6, 1))], True),
    (2, 3, [(1, (3, 3))], False),
    (3, 1, [(1, (2, 0, 0)), (1, (0, 3, 0)), (1, (1, 1, 0))], True),
    (3, 1, [(1, (1, 1, 1))], False),
    (3, 2, [(1, (1, 3, 4)), (1, (4, 1, 2))], True),
    (3, 2, [(1, (2, 2, 2))], False),
    (1, 2, [(1, (1,))], True),
    (1, 2, [(1, (2,))], False),
    (1, 4, [(1, (3,))], True),
])
def test_theorem1_polynomial_exactness(oracle, case):
    """Theorem 1: the n-layer value equals the surface through T^n; hence on
    original values it reproduces any polynomial each of whose monomials has
    some exponent below n (proof, Sec. III-A), and not i^n j^n."""
    ndim, n, monos, exact = case
    shape = {1: (12,), 2: (9, 10), 3: (7, 8, 9)}[ndim]
    f = _poly_field(shape, monos)
    assert np.abs(f).max() < 2 ** 40  # exact in float64
    pred = oracle.predict_original(f, layers=n)
    inner = _interior(shape, n)
    resid = (pred - f)[inner]
    if exact:
        assert np.all(resid == 0)
    else:
        assert np.any(resid != 0)


def test_zero_halo_first_row_is_lower_dimensional(oracle):
    """Reading: outside neighbours are zero, so for n = 1 the first row of a 2D
    array is predicted by the 1D Lorenzo rule and the first point by 0."""
    f = np.arange(1, 13, dtype=np.float64).reshape(3, 4) ** 2
    pred = oracle.predict_original(f, layers=1)
    assert pred[0, 0] == 0
    assert np.all(pred[0, 1:] == f[0, :-1])
    assert np.all(pred[1:, 0] == f[:-1, 0])


# ----------------------------------------------------- hand-worked examples


def test_hand_2x2(oracle):
    g = golden("hand_2x2_lorenzo.txt")
    x = np.array([float(v) for v in g["x"][0]], np.float32).reshape(2, 2)
    eb = float(g["eb"][0][0])
    c3, xp3, nu3 = oracle.quantize(x, m=3, eb_mode="abs", eb_abs=eb)
    assert c3.ravel().tolist() == [int(v) for v in g["m3_codes"][0]] and nu3 == 0
    assert np.array_equal(xp3, x)
    c2, xp2, nu2 = oracle.quantize(x, m=2, eb_mode="abs", eb_abs=eb)
    assert c2.ravel().tolist() == [int(v) for v in g["m2_codes"][0]] and nu2 == 2
    assert xp2.ravel().tolist() == [float(v) for v in g["m2_xprime"][0]]


def _container_words(buf, off_field, count):
    off = int.from_bytes(buf[off_field:off_field + 8], "little")
    return [int.from_bytes(buf[off + 4 * i: off + 4 * i + 4], "little") for i in range(count)]


HDR = {"off_cb": 136, "off_ch": 144, "off_bs": 152, "off_hd": 160, "off_tl": 168}


def test_hand_1d_bitstream(oracle):
    g = golden("hand_1d_bitstream.txt")
    x = np.zeros(64, np.float32)
    x[2] = x[3] = 1.0
    codes, _, _ = oracle.quantize(x, m=2, eb_mode="abs", eb_abs=0.5)
    assert codes[:8].tolist() == [int(v) for v in g["codes_head"][0]]
    h = np.bincount(codes, minlength=4)
    lens = oracle.huffman_lengths(h)
    assert lens.tolist() == [0, 2, 1, 2]
    buf, st = oracle.compress(x, m=2, eb_mode="abs", eb_abs=0.5)
    assert st["raw_fallback"] == 0
    assert st["huff_bits"] == int(g["huff_bits"][0][0])
    words = _container_words(buf, HDR["off_bs"], 3)
    assert words == [int(g["word0"][0][0], 16), int(g["word1"][0][0], 16), int(g["word2"][0][0], 16)]
    assert _container_words(buf, HDR["off_ch"], 1) == [int(g["chunk_bits"][0][0])]
    # codebook: (u16 sym, u8 len) sorted by symbol
    off = int.from_bytes(buf[136:144], "little")
    cb = [struct.unpack_from("<HB", buf, off + 3 * i) for i in range(3)]
    assert cb == [(1, 2), (2, 1), (3, 2)]
    assert np.array_equal(oracle.decompress(buf), x)


def test_chunk_half_offsets(oracle):
    """Reading A17: after the u32 bit counts, the chunk table holds for each
    chunk the bits of its first C/2 codes (all of them in a chunk of at most
    C/2 codes).  Recomputed here from the codes and the code lengths of the
    container's codebook; a wrong entry is rejected by the decompressor."""
    C = 256
    for n in (640, 700, 1024):
        x = np.cumsum(F.rng(7).normal(0, 1, n)).astype(np.float32)
        buf, st, codes, _ = oracle.compress(x, debug=True, m=6, eb_mode="abs", eb_abs=0.05, chunk=C)
        assert st["raw_fallback"] == 0
        nc = int.from_bytes(buf[128:136], "little")
        assert nc == (n + C - 1) // C
        off_cb = int.from_bytes(buf[136:144], "little")
        off_ch = int.from_bytes(buf[144:152], "little")
        n_used = int.from_bytes(buf[124:128], "little")
        lens = np.zeros(1 << 6, np.int64)
        for i in range(n_used):
            sym, ln = struct.unpack_from("<HB", buf, off_cb + 3 * i)
            lens[sym] = ln
        bits = lens[codes.astype(np.int64)]
        for c in range(nc):
            lo, hi = c * C, min(n, (c + 1) * C)
            total = int.from_bytes(buf[off_ch + 4 * c: off_ch + 4 * c + 4], "little")
            half = int.from_bytes(buf[off_ch + 4 * nc + 2 * c: off_ch + 4 * nc + 2 * c + 2], "little")
            assert total == int(bits[lo:hi].sum())
            assert half == int(bits[lo:min(hi, lo + C // 2)].sum())
        assert np.max(np.abs(oracle.decompress(buf).astype(np.float64) - x)) < 0.05
        bad = bytearray(buf)
        pos = off_ch + 4 * nc
        bad[pos] = (bad[pos] + 1) & 0xFF
        with pytest.raises(oracle.OracleError):
            oracle.decompress(bytes(bad))


def test_hand_1d_unpredictable(oracle):
    g = golden("hand_1d_unpred.txt")
    x = np.zeros(128, np.float32)
    x[2] = x[3] = np.float32(5.3)
    assert struct.unpack("<I", struct.pack("<f", x[2]))[0] == 0x40A9999A
    buf, st = oracle.compress(x, m=2, eb_mode="abs", eb_abs=0.5)
    assert st["raw_fallback"] == 0
    assert st["n_unpred"] == int(g["n_unpred"][0][0])
    assert st["huff_bits"] == int(g["huff_bits"][0][0])
    bsw = _container_words(buf, HDR["off_bs"], 4)
    assert bsw[0] == int(g["bs_word0"][0][0], 16)
    assert bsw[1] == int(g["bs_word1"][0][0], 16)
    assert bsw[3] == int(g["bs_word3"][0][0], 16)
    assert _container_words(buf, HDR["off_hd"], 1) == [int(g["heads_word0"][0][0], 16)]
    assert st["tail_bits"] == int(g["tail_bits"][0][0])
    assert _container_words(buf, HDR["off_tl"], 1) == [int(g["tails_word0"][0][0], 16)]
    out = oracle.decompress(buf)
    assert out[:6].tolist() == [float(v) for v in g["decompressed_head"][0]]
    assert np.all(np.abs(out.astype(np.float64) - x) < 0.5)


# ------------------------------------------------- quantization brute force


def _exact_pred(xp, idx, coefs, koffs):
    p = Fraction(0)
    for c, k in zip(coefs, koffs):
        src = tuple(i - kk for i, kk in zip(idx, k))
        if all(s >= 0 for s in src):
            p += int(c) * Fraction(float(xp[src]))
    return p


@pytest.mark.parametrize("seed", range(6))
def test_quantization_brute_force(oracle, seed):
    """Sec. IV-A: the 2^m - 1 intervals of width 2eb around p + 2k eb are
    disjoint, so at most one k covers x.  On small dyadic inputs (all float
    arithmetic exact) enumerate every k in exact rational arithmetic."""
    rng = np.random.default_rng(seed)
    ndim = 1 + seed % 3
    shape = {1: (17,), 2: (5, 6), 3: (3, 4, 5)}[ndim]
    n = 1 + seed % 2
    m = 2 + seed % 3
    x = (rng.integers(-40, 40, size=shape) / 8.0).astype(np.float32)
    eb = [0.25, 0.5, 1.0][seed % 3]
    codes, xp, nu = oracle.quantize(x, m=m, layers=n, eb_mode="abs", eb_abs=eb)
    coefs, koffs = oracle.coefficients(ndim, n)
    half = 1 << (m - 1)
    ebq = Fraction(eb)
    unpred = 0
    for idx in itertools.product(*[range(s) for s in shape]):
        p = _exact_pred(xp, idx, coefs, koffs)
        xv = Fraction(float(x[idx]))
        valid = [k for k in range(-(half - 1), half) if abs(xv - (p + 2 * k * ebq)) < ebq]
        assert len(valid) <= 1
        if valid:
            assert codes[idx] == valid[0] + half
            assert Fraction(float(xp[idx])) == p + 2 * valid[0] * ebq
        else:
            assert codes[idx] == 0
            unpred += 1
            assert abs(Fraction(float(xp[idx])) - xv) < ebq
    assert unpred == nu


def test_m1_is_the_single_interval_hit_rate(oracle):
    """Sec. III-B defines R_PH with one interval: predictable iff the
    prediction (from decompressed values) is within eb.  With m = 1 the only
    code besides 0 is the centre."""
    rng = np.random.default_rng(3)
    x = np.cumsum(rng.normal(0, 1, 400)).astype(np.float64).reshape(20, 20)
    eb = 0.7
    codes, xp, nu = oracle.quantize(x, m=1, eb_mode="abs", eb_abs=eb)
    coefs, koffs = oracle.coefficients(2, 1)
    for idx in itertools.product(range(20), range(20)):
        p = float(_exact_pred(xp, idx, coefs, koffs))
        predictable = abs(x[idx] - p) < eb
        assert (codes[idx] == 1) == predictable


def test_prediction_uses_decompressed_values(oracle):
    """Sec. III-B / Algorithm 1: predictions read preceding decompressed
    values, so codes differ from those computed from original values."""
    rng = np.random.default_rng(5)
    x = (np.cumsum(rng.normal(0, 0.3, 4096))).astype(np.float32).reshape(64, 64)
    eb = 0.05
    codes, xp, _ = oracle.quantize(x, m=8, eb_mode="abs", eb_abs=eb)
    porig = oracle.predict_original(x)
    korig = np.rint((x - porig) / (2 * eb))
    assert np.any(codes.astype(np.int64) - 128 != korig)


# ------------------------------------------------------------ invariants


FIELDS = [
    ("smooth3d", lambda: __import__("fieldgen").smooth3d((24, 20, 36))),
    ("climate2d", lambda: __import__("fieldgen").climate2d((60, 90))),
    ("walk1d", lambda: np.cumsum(np.random.default_rng(1).normal(0, 1, 5000)).astype(np.float32)),
]


@pytest.mark.parametrize("name,make", FIELDS)
@pytest.mark.parametrize("n", [1, 2, 3, 4])
@pytest.mark.parametrize("ebrel", [1e-2, 1e-4, 1e-6])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_error_bound_and_roundtrip(oracle, name, make, n, ebrel, dtype):
    """Metric 1: |x - x'| < eb at every point; the decompressor reproduces the
    compressor's recorded values bit for bit; BR * CF = 32 / 64."""
    x = make().astype(dtype)
    buf, st, codes, xp = oracle.compress(x, debug=True, layers=n, m=0, eb_mode="rel", eb_rel=ebrel)
    out = oracle.decompress(buf)
    if st["raw_fallback"]:
        assert np.array_equal(out.view(np.uint8), x.view(np.uint8))
    else:
        assert np.array_equal(out.view(np.uint8), xp.view(np.uint8))
    ebT = st["eb_used"]
    err = np.abs(out.astype(np.float64) - x.astype(np.float64))
    assert np.all(err < ebT)
    assert ebT <= ebrel * (float(x.max()) - float(x.min()))
    bits = 32 if dtype == np.float32 else 64
    br = len(buf) * 8 / x.size
    cf = x.nbytes / len(buf)
    assert abs(br * cf - bits) < 1e-9
    h = np.bincount(codes.ravel(), minlength=1 << st["m_used"])
    assert h.sum() == x.size and h[0] == st["n_unpred"]
    assert abs(st["hit_rate"] - (1 - h[0] / x.size)) < 1e-12


def test_truncation_keeps_exponent_gap_bits(oracle):
    """Unpredictable storage: sign, exponent and r = e(x) - e(eb) mantissa
    bits are kept, so the error is below 2^E(eb) <= eb."""
    rng = np.random.default_rng(9)
    x = rng.normal(0, 1000, 3000).astype(np.float32)
    eb = 0.01
    codes, xp, nu = oracle.quantize(x, m=1, eb_mode="abs", eb_abs=eb, block=[1])
    assert nu > 2500
    ue = (struct.unpack("<I", struct.pack("<f", np.float32(eb)))[0] >> 23) & 255
    for xi, xpi, c in zip(x, xp, codes):
        if c:
            continue
        b = struct.unpack("<I", struct.pack("<f", xi))[0]
        e = (b >> 23) & 255
        kept = struct.unpack("<I", struct.pack("<f", xpi))[0]
        if e < ue:
            assert kept & 0x7FFFFFFF == 0
        else:
            r = min(e - ue, 23)
            assert kept == b & ~((1 << (23 - r)) - 1)
        assert abs(float(xi) - float(xpi)) < 2.0 ** (ue - 127) <= eb


def test_nonfinite(oracle):
    x = np.linspace(0, 1, 1000).astype(np.float32)
    x[10] = np.nan
    x[500] = np.inf
    with pytest.raises(oracle.OracleError) as e:
        oracle.compress(x, eb_mode="rel", eb_rel=1e-3)
    assert e.value.code == oracle.ENONFINITE
    buf, st = oracle.compress(x, eb_mode="abs", eb_abs=1e-3)
    out = oracle.decompress(buf)
    assert np.isnan(out[10]) and out[500] == np.inf
    fin = np.isfinite(x)
    assert np.all(np.abs(out[fin] - x[fin]) < 1e-3)


def test_zero_bound_is_lossless(oracle):
    x = np.random.default_rng(2).normal(0, 1, (30, 40)).astype(np.float32)
    x[0, 0] = np.float32(1e-40)  # subnormal survives
    buf, st = oracle.compress(x, eb_mode="abs", eb_abs=0.0)
    assert np.array_equal(oracle.decompress(buf).view(np.uint32), x.view(np.uint32))


def test_raw_fallback(oracle):
    x = np.random.default_rng(4).normal(0, 1, 4096).astype(np.float32)
    buf, st = oracle.compress(x, eb_mode="abs", eb_abs=1e-30)
    assert st["raw_fallback"] == 1
    assert len(buf) == 192 + x.nbytes
    assert np.array_equal(oracle.decompress(buf).view(np.uint32), x.view(np.uint32))


def test_blocks_are_independent(oracle):
    """Reading: neighbours outside an independent block read as zero, so
    compressing a block alone gives the same codes as inside the array."""
    x = __import__("fieldgen").smooth3d((16, 24, 20)).astype(np.float32)
    blk = [8, 12, 10]
    codes, _, _ = oracle.quantize(x, m=8, eb_mode="abs", eb_abs=1e-3, block=blk)
    sub = np.ascontiguousarray(x[8:16, 12:24, 10:20])
    csub, _, _ = oracle.quantize(sub, m=8, eb_mode="abs", eb_abs=1e-3)
    assert np.array_equal(codes[8:16, 12:24, 10:20], csub)


def test_adaptive_m_rule(oracle):
    """Sec. IV-B: the smallest m whose intervals cover theta of the points in
    the 2^16-code run (theta = 0.9)."""
    x = __import__("fieldgen").climate2d((90, 120))
    ebabs = 1e-4 * float(x.max() - x.min())
    c16, _, _ = oracle.quantize(x, m=16, eb_mode="abs", eb_abs=ebabs)
    k = c16.astype(np.int64).ravel()
    k = k[k != 0] - 32768
    want = 16
    for m in range(1, 17):
        if np.sum(np.abs(k) <= (1 << (m - 1)) - 1) >= 0.9 * x.size:
            want = m
            break
    buf, st = oracle.compress(x, m=0, eb_mode="abs", eb_abs=ebabs)
    assert st["m_used"] == want
    assert oracle.inspect(buf)["m_used"] == want


def test_corrupt_streams_are_rejected(oracle):
    x = __import__("fieldgen").smooth3d((16, 16, 16))
    buf, st = oracle.compress(x, eb_mode="rel", eb_rel=1e-4)
    assert oracle.decompress_raw(buf, x.nbytes) == 0
    assert oracle.decompress_raw(buf, x.nbytes - 4) == oracle.ECAPACITY
    assert oracle.decompress_raw(buf[:100], x.nbytes) == oracle.ECORRUPT
    assert oracle.decompress_raw(buf[:-8], x.nbytes) == oracle.ECORRUPT
    bad = bytearray(buf)
    bad[0] ^= 1
    assert oracle.decompress_raw(bytes(bad), x.nbytes) == oracle.ECORRUPT
    rng = np.random.default_rng(0)
    for _ in range(20):
        bad = bytearray(buf)
        pos = int(rng.integers(192, len(buf)))
        bad[pos] ^= 1 << int(rng.integers(0, 8))
        rc = oracle.decompress_raw(bytes(bad), x.nbytes)
        assert rc in (0, oracle.ECORRUPT)


# -------------------------------------------------------------- Huffman


def _kraft_min_cost(freq, maxlen=8):
    best = None
    for lens in itertools.product(range(1, maxlen + 1), repeat=len(freq)):
        if sum(Fraction(1, 2 ** l) for l in lens) <= 1:
            cost = sum(f * l for f, l in zip(freq, lens))
            best = cost if best is None else min(best, cost)
    return best


@pytest.mark.parametrize("seed", range(12))
def test_huffman_lengths_optimal_by_enumeration(oracle, seed):
    rng = np.random.default_rng(seed)
    s = 2 + seed % 5
    freq = rng.integers(1, 30, size=s).tolist()
    if seed % 4 == 0:
        freq = [5] * s  # all ties
    full = [0] * 3 + freq  # unused symbols get no code
    lens = oracle.huffman_lengths(full)[3:]
    assert all(l >= 1 for l in lens)
    assert sum(Fraction(1, 2 ** int(l)) for l in lens) == 1  # full binary tree
    cost = sum(f * int(l) for f, l in zip(freq, lens))
    assert cost == _kraft_min_cost(freq, maxlen=s)
    # total cost = sum of internal-node weights (independent heap construction)
    h = list(freq)
    heapq.heapify(h)
    internal = 0
    while len(h) > 1:
        a, b = heapq.heappop(h), heapq.heappop(h)
        internal += a + b
        heapq.heappush(h, a + b)
    assert cost == internal


def test_huffman_tie_rule_hand_example(oracle):
    g = golden("hand_huffman_ties.txt")
    freq = [int(v) for v in g["freq"][0]]
    assert oracle.huffman_lengths(freq).tolist() == [int(v) for v in g["len"][0]]


def test_huffman_single_symbol(oracle):
    assert oracle.huffman_lengths([0, 0, 7, 0]).tolist() == [0, 0, 1, 0]


def test_huffman_length_limit(oracle):
    """Fibonacci frequencies make a degenerate tree deeper than 27 bits; the
    halving rule brings it back under the limit and stays decodable."""
    fib = [1, 1]
    while len(fib) < 40:
        fib.append(fib[-1] + fib[-2])
    lens = oracle.huffman_lengths(fib)
    assert lens.max() <= 27
    assert sum(Fraction(1, 2 ** int(l)) for l in lens) <= 1


def test_canonical_codes_prefix_free_roundtrip(oracle):
    """Many symbols (m = 12) with a wide spread of k survive the round trip."""
    rng = np.random.default_rng(8)
    x = np.cumsum(rng.standard_cauchy(20000) * 0.01).astype(np.float64)
    buf, st = oracle.compress(x, m=12, eb_mode="abs", eb_abs=1e-4)
    assert st["n_used_syms"] > 200
    out = oracle.decompress(buf)
    assert np.all(np.abs(out - x) < 1e-4)


def test_fibonacci_field_forces_the_length_limit(oracle):
    """The full-size GPU case of the A14 rebuild: its 1D field has exact
    codes k_i + 2^(m-1) with Fibonacci counts, a textbook Huffman tree of
    those counts is 28 levels deep (beyond the 27-bit limit), and the
    oracle's codebook comes out within the limit after the rebuild."""
    import heapq
    from test_gpu_fullsize import fibonacci_field
    x, fib = fibonacci_field(29, np.float32, 20170662)
    # textbook Huffman depth by a heap of (weight, depth) pairs
    heap = [(f, 0) for f in fib]
    heapq.heapify(heap)
    while len(heap) > 1:
        a, b = heapq.heappop(heap), heapq.heappop(heap)
        heapq.heappush(heap, (a[0] + b[0], max(a[1], b[1]) + 1))
    assert heap[0][1] == 28
    codes, xp, nu = oracle.quantize(x, m=8, layers=1, eb_mode="abs", eb_abs=0.5)
    assert nu == 0 and np.array_equal(xp, x)
    counts = np.bincount(codes.ravel(), minlength=256)
    assert sorted(counts[counts > 0].tolist()) == sorted(fib)
    buf, st = oracle.compress(x, layers=1, m=8, eb_mode="abs", eb_abs=0.5)
    off_cb = int.from_bytes(buf[136:144], "little")
    cb = np.frombuffer(buf[off_cb:off_cb + 3 * st["n_used_syms"]], np.uint8).reshape(-1, 3)
    lens = cb[:, 2].astype(np.int64)
    assert lens.max() <= 27 and np.sum(2.0 ** -lens) <= 1.0
    assert np.array_equal(oracle.decompress(buf), x)


def test_hand_xor_unpredictable(oracle):
    """The XOR coding of unpredictable values against the hand-worked records
    of tests/golden/hand_xor_unpred.txt: the per-chunk bit table in the heads
    section, the records in the tails section, flag bit 1, and the
    reconstruction (the same values as the plain coding)."""
    g = golden("hand_xor_unpred.txt")
    x = np.zeros(512, np.float32)
    x[10:13] = [100.0, 100.25, 100.5]
    x[13:300] = 100.5
    x[300] = 100.0
    x[301:317] = 100.0 - 0.125 * np.arange(1, 17)
    x[317] = 100.0
    kw = dict(m=2, eb_mode="abs", eb_abs=0.0625, chunk=256)
    buf, st = oracle.compress(x, unpred_coding=1, **kw)
    plain, sp = oracle.compress(x, **kw)
    assert st["raw_fallback"] == 0 and st["n_unpred"] == int(g["n_unpred"][0][0]) == sp["n_unpred"]
    assert struct.unpack("<H", buf[6:8])[0] == 2
    bits = "".join("".join(r) for r in g["record"])
    assert st["tail_bits"] == len(bits) == 73
    table = _container_words(buf, HDR["off_hd"], 2)
    assert table == [int(v) for v in g["chunk_bits"][0]]
    nw = (len(bits) + 31) // 32
    want = [int(bits[32 * i:32 * i + 32].ljust(32, "0"), 2) for i in range(nw)]
    assert _container_words(buf, HDR["off_tl"], nw) == want
    out = oracle.decompress(buf)
    assert np.array_equal(out.view(np.uint32), oracle.decompress(plain).view(np.uint32))
    assert out[10:15].tolist() == [100.0, 100.25, 100.5, 100.5, 100.5] and out[318] == 0.0
    assert out[317] == 100.0 and np.all(np.abs(out.astype(np.float64) - x) < 0.0625)
    assert oracle.inspect(buf)["unpred_coding"] == 1


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_xor_coding_round_trip_and_bound(oracle, dtype):
    """Both codings of unpredictable values reconstruct the same values (the
    XOR coding only re-encodes the reduced patterns), within the bound, on
    fields with many unpredictable points, non-finite values in ABS mode and a
    lossless bound."""
    import fieldgen as F
    rng = np.random.default_rng(21)
    cases = [
        (np.cumsum(rng.normal(0, 30, 6000)).astype(dtype), dict(m=4, eb_mode="rel", eb_rel=1e-4)),
        (F.climate2d((60, 80)).astype(dtype), dict(m=8, eb_mode="rel", eb_rel=1e-6, layers=2)),
        (F.smooth3d((12, 14, 16)).astype(dtype), dict(m=0, eb_mode="abs", eb_abs=1e-5, chunk=512)),
        (rng.normal(0, 1, 3000).astype(dtype), dict(m=8, eb_mode="abs", eb_abs=0.0)),
    ]
    spiky = np.cumsum(rng.normal(0, 1, 4000)).astype(dtype)
    spiky[[5, 77, 900]] = [np.nan, np.inf, -np.inf]
    cases.append((spiky, dict(m=6, eb_mode="abs", eb_abs=1e-2)))
    for x, kw in cases:
        a, sa = oracle.compress(x, **kw)
        b, sb, _, xp = oracle.compress(x, debug=True, unpred_coding=1, **kw)
        assert sa["n_unpred"] == sb["n_unpred"] > 0
        ya, yb = oracle.decompress(a), oracle.decompress(b)
        u = np.uint32 if dtype == np.float32 else np.uint64
        # a container that would not be smaller than the field is a raw copy
        for y, s in ((ya, sa), (yb, sb)):
            assert np.array_equal(y.view(u), (x if s["raw_fallback"] else xp).view(u))
        fin = np.isfinite(x)
        eb = sb["eb_used"]
        if eb > 0:
            assert np.all(np.abs(yb[fin].astype(np.float64) - x[fin]) < eb)
        else:
            assert np.array_equal(yb.view(u), x.view(u))
