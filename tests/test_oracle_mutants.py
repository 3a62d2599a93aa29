"""The oracle's pins must catch plausible mistakes (CPU only).

Each case plants one mistake in a temporary copy of the oracle source,
builds it, and runs the fast pin tests against it: they must fail.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    "coefficient sign": ("szref.c", "if (coef) coef[count] = -prod;", "if (coef) coef[count] = prod;"),
    "dropped term": ("szref_traverse.inc", "for (int t = 0; t < S->nterms; t++) {",
                     "for (int t = 0; t < S->nterms - 1; t++) {"),
    "transposed operand": ("szref_traverse.inc", "src += (c[d] - (uint64_t)k[d]) * L->stride[d];",
                           "src += (c[d] - (uint64_t)k[2 - d]) * L->stride[d];"),
    "truncating rounding": ("szref.c", "static float rint_f32(float v) { return rintf(v); }",
                            "static float rint_f32(float v) { return truncf(v); }"),
    "bound not strict": ("szref_traverse.inc", "if (!(err < ebT)) return 0;", "if (!(err <= ebT + ebT)) return 0;"),
    "huffman tie rule": ("szref.c", "if (i < s && (j >= next || w[i] <= w[j])) pick[q] = i++;",
                         "if (i < s && (j >= next || w[i] < w[j])) pick[q] = i++;"),
    "bit order": ("szref.c", "w->words[b >> 5] |= 1u << (31 - (b & 31));", "w->words[b >> 5] |= 1u << (b & 31);"),
    "kept mantissa bits": ("szref_traverse.inc", "r = e - e_eb;\n    if (r > MANT) r = MANT;",
                           "r = e - e_eb - 1;\n    if (r < 0) r = 0;\n    if (r > MANT) r = MANT;"),
    "xor reference kept across chunks": (
        "szref_traverse.inc",
        "  for (uint64_t c = 0; c * C < n; c++) {\n    const uint64_t before = recs->nbits;\n    UT prev = 0;",
        "  UT prev = 0;\n  for (uint64_t c = 0; c * C < n; c++) {\n    const uint64_t before = recs->nbits;"),
    "xor leading byte cap": ("szref_traverse.inc", "while (lzb < BMAX &&", "while (lzb <= BMAX &&"),
    "xor record length": ("szref_traverse.inc", "const int nb = q - 8 * lzb;", "const int nb = q - 8 * lzb + 1;"),
    "chunk half offset": ("szref.c", "if (i % C < C / 2) chunk_mid", "if (i % C <= C / 2) chunk_mid"),
}

FAST = ("table1 or lorenzo or finite_difference or theorem1 or hand or brute or m1_ or "
        "truncation or tie_rule or half_offsets")


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    fname, old, new = MUTANTS[name]
    src = os.path.join(ROOT, "oracle")
    for f in ("szref.c", "szref.h", "szref_traverse.inc"):
        shutil.copy(os.path.join(src, f), tmp_path / f)
    text = (tmp_path / fname).read_text()
    assert old in text, f"mutation site for {name!r} not found"
    (tmp_path / fname).write_text(text.replace(old, new, 1))
    so = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-o",
                    str(so), str(tmp_path / "szref.c"), "-lm"], check=True)
    env = dict(os.environ, SZREF_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-k", FAST],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"planted mistake {name!r} passed every pin:\n{r.stdout[-2000:]}"
