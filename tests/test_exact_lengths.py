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
    assert [e[0] for e in cols] == g.smooth5(8, 512)
    assert [e[0] for e in rows] == g.smooth5(4, 256)
    for e in cols:
        L, t, tx, rad = e[0], e[1], e[2], e[3:]
        assert rad == g.radices(L) and t == g.col_threads(L) and tx == 16
    for e in rows:
        M, wpb, rpw, rad = e[0], e[1], e[2], e[3:]
        assert rad == g.radices(M, big=8) and wpb == 4 and rpw == g.row_rows(M)
        assert 16 not in rad


def test_radix_products_and_limits():
    for macro in ("MVD_EXACT_COL", "MVD_EXACT_ROW"):
        for e in _entries(macro):
            L, rad = e[0], e[3:]
            prod = 1
            for r in rad:
                assert r in (2, 3, 4, 5, 8, 16)
                prod *= r
            assert prod == L
    for e in _entries("MVD_EXACT_COL"):
        L, t, tx = e[:3]
        assert t % 64 == 0 and t <= 1024
        assert tx * L * 8 + L * 8 <= 160 * 1024  # tile and twiddles fit the LDS
    for e in _entries("MVD_EXACT_ROW"):
        M, wpb, rpw = e[:3]
        assert wpb * rpw * M * 8 + 2 * M * 8 <= 64 * 1024  # rows and twiddle tables in LDS
        assert rpw * (M // max(e[3:])) >= 64 or rpw == 16  # the largest-radix stage fills a wave
