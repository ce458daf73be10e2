"""The committed list of per-length compile-time plans is what its generator
writes, every radix sequence multiplies to its length with supported radices,
and every 5-smooth length in the covered ranges has a plan."""
import importlib.util
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1308_0730_amd", "csrc")


def _gen():
    spec = importlib.util.spec_from_file_location("gen_exact_lengths", os.path.join(CSRC, "gen_exact_lengths.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def _entries(macro):
    txt = open(os.path.join(CSRC, "mvd_exact_lengths.h")).read()
    body = txt.split(f"#define {macro}(X)")[1].split("\n\n")[0]
    return [list(map(int, m.split(","))) for m in re.findall(r"X\(([0-9, ]+)\)", body)]


def test_header_matches_generator(tmp_path):
    g = _gen()
    cols = _entries("MVD_EXACT_COL")
    rows = _entries("MVD_EXACT_ROW")
    assert [e[0] for e in cols] == g.smooth5(8, g.MAX_COL)
    assert [e[0] for e in rows] == g.smooth5(4, g.MAX_ROW)
    for e in cols:
        L, t, tx, rad = e[0], e[1], e[2], e[3:]
        assert rad == g.radices(L) and t == g.col_threads(L) and tx == g.col_lines(L) == (16 if L <= 512 else 8)
    for e in rows:
        M, wpb, rpw, rad = e[0], e[1], e[2], e[3:]
        assert rad == g.row_radices(M) and wpb == 4 and rpw == g.row_rows(M)
        assert 16 not in rad


def test_radix_products_and_limits():
    for macro in ("MVD_EXACT_COL", "MVD_EXACT_ROW"):
        for e in _entries(macro):
            L, rad = e[0], e[3:]
            prod = 1
            for r in rad:
                assert r in (2, 3, 4, 5, 8, 16) + _gen().COMPOSITE
                prod *= r
            assert prod == L
    for e in _entries("MVD_EXACT_COL"):
        L, t, tx = e[:3]
        assert t % 64 == 0 and t <= 1024
        assert tx * L * 8 + L * 8 <= 160 * 1024  # tile and twiddles fit the LDS
    for e in _entries("MVD_EXACT_ROW"):
        M, wpb, rpw = e[:3]
        assert wpb * rpw * M * 8 <= _gen().ROW_LDS  # rows of a workgroup within the LDS budget
        # the largest-radix stage fills a wave unless 16 rows or the LDS budget stop it
        assert rpw * (M // max(e[3:])) >= 64 or rpw == 16 or wpb * (rpw + 1) * M * 8 > _gen().ROW_LDS


def test_composite_twiddle_header():
    """fft_small_tw.h holds cos and sin of 2 pi m / R for every composite
    radix, as the generator computes them."""
    import math
    g = _gen()
    txt = open(os.path.join(CSRC, "fft_small_tw.h")).read()
    for R in g.COMPOSITE:
        body = txt.split(f"struct SmallTw<{R}> {{")[1].split("\n};")[0]
        c = [float(x.rstrip("f")) for x in re.search(r"c\[\d+\] = \{([^}]*)\}", body).group(1).split(",")]
        s = [float(x.rstrip("f")) for x in re.search(r"s\[\d+\] = \{([^}]*)\}", body).group(1).split(",")]
        assert len(c) == len(s) == R
        for m in range(R):
            assert abs(c[m] - math.cos(2 * math.pi * m / R)) < 1e-15
            assert abs(s[m] - math.sin(2 * math.pi * m / R)) < 1e-15


def test_composite_decomposition_algebra():
    """The R1 x R2 register butterfly's index map and twiddles (inputs
    x[R2 n1 + n2], inner DFTs over n1, twiddle exp(-2 pi i n2 k1 / R), outer
    DFTs over n2, output X[k1 + R1 k2]) give the R-point DFT."""
    import numpy as np
    rng = np.random.default_rng(0)
    for R in _gen().COMPOSITE:
        for R1 in range(2, R):
            if R % R1:
                continue
            R2 = R // R1
            x = rng.normal(size=R) + 1j * rng.normal(size=R)
            a = np.empty((R2, R1), complex)
            for n2 in range(R2):
                t = np.fft.fft(x[n2::R2])  # x[R2 n1 + n2] over n1
                a[n2] = t * np.exp(-2j * np.pi * n2 * np.arange(R1) / R)
            X = np.empty(R, complex)
            for k1 in range(R1):
                X[k1 + R1 * np.arange(R2)] = np.fft.fft(a[:, k1])
            assert np.allclose(X, np.fft.fft(x), atol=1e-12)



def test_column_length_classes():
    """Every column length belongs to exactly one class; a class has one
    thread count (that of each member's own plan) and the longest member as
    its LDS size; the class lists carry each length's own radices."""
    g = _gen()
    txt = open(os.path.join(CSRC, "mvd_exact_lengths.h")).read()
    of = dict(_entries("MVD_COL_CLASS_OF"))
    assert sorted(of) == g.smooth5(8, g.MAX_COL)
    body = txt.split("#define MVD_COL_CLASSES(X)")[1].split("\n\n")[0]
    seen = []
    for line in body.splitlines()[1:]:
        m = re.match(r"\s*X\((\d+), (\d+), (\d+), (\d+), (.*)\)( \\)?$", line)
        assert m, line
        c, t, tx, lmax = int(m.group(1)), int(m.group(2)), int(m.group(3)), int(m.group(4))
        plans = [list(map(int, p.split(","))) for p in re.findall(r"ColPlan<([0-9, ]+)>", m.group(5))]
        lens = [p[0] for p in plans]
        assert lmax == max(lens)
        for p in plans:
            L = p[0]
            assert of[L] == c == g.col_class(L)
            assert t == g.col_threads(L) and tx == g.col_lines(L)
            assert p[1:] == g.radices(L)
        seen += lens
    assert sorted(seen) == g.smooth5(8, g.MAX_COL)
