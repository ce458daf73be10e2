"""Writes mvd_exact_lengths.h: the lengths that get compile-time transform
plans, with their radix sequences and launch shapes, and fft_small_tw.h: the
constant twiddles of the composite radices.

Radices: the power-of-two part as 16s (columns) or 8s (rows), then one 8, 4
or 2 (512 as 8 x 8 x 8 for columns; a final 2 after a 16 or an 8 split as
8 x 4 or 4 x 4); then the odd part, 5s then 3s.  Columns merge further: a
trailing 2 or 4 with the first odd factor (2 x 3 = 6, 2 x 5 = 10, 4 x 3 = 12,
4 x 5 = 20), and the remaining odd factors in pairs (5 x 5 = 25, 5 x 3 = 15,
3 x 3 = 9).  A composite radix is one register butterfly (an R1 x R2
decomposition with constant twiddles), so a 5-smooth column takes two or
three LDS stages instead of up to five.  Rows keep the small radices: a
wave-local row transform has no workgroup barrier between stages, and the
extra rows per wave that a large radix needs to fill the lanes raise the
fused row epilogues' register use (up to 256 VGPRs: one wave per SIMD).
Column passes (y, z): every 5-smooth length in [8, 1024]; tiles of 16 lines
(128-byte row segments) up to 512 points and of 8 lines above; threads 64,
128, 256 or 512 by length (512 points on 256 threads).
Column length classes (lengths up to 48, 128, 256, between 256 and 512, 512,
and above 512), each of one thread count and tile, for the kernels that serve blocks of several
lengths in one launch.
Row passes (x): every 5-smooth half-row length M in [4, 1024]; four waves per
workgroup; each wave owns ceil(64 * largest radix / M) rows, so the
largest-radix stage has a butterfly for nearly every lane, and where that
is not exactly one round of butterflies at least 512 complex values (at most
16 rows, and at most 32 KB of rows per workgroup).
"""
import math
import os


def smooth5(lo, hi):
    out = []
    for n in range(lo, hi + 1):
        m = n
        for p in (2, 3, 5):
            while m % p == 0:
                m //= p
        if m == 1:
            out.append(n)
    return out


def radices(n, big=16, merge=True):
    r = []
    p2 = 0
    while n % 2 == 0:
        n //= 2
        p2 += 1
    if p2 == 9 and big == 16:
        r += [8, 8, 8]
        p2 = 0
    step = 4 if big == 16 else 3
    while p2 >= step:
        r.append(1 << step)
        p2 -= step
    if p2 == 1 and r:  # a lone radix-2 stage: 16 x 2 -> 8 x 4, 8 x 2 -> 4 x 4
        r[-1] //= 2
        p2 = 2
    if p2:
        r.append(1 << p2)
    odd = []
    for p in (5, 3):
        while n % p == 0:
            odd.append(p)
            n //= p
    assert n == 1
    if merge and odd and r and r[-1] in (2, 4):
        r[-1] *= odd.pop(0)
    while merge and len(odd) >= 2:
        r.append(odd.pop(0) * odd.pop(0))
    return r + odd


COMPOSITE = (6, 9, 10, 12, 15, 20, 25)


def unit(m, R):
    """(cos, sin) of 2 pi m / R: exact at multiples of a quarter turn, and
    from the reduced angle otherwise so that symmetric entries are equal."""
    if (4 * m) % R == 0:
        return [(1.0, 0.0), (0.0, 1.0), (-1.0, 0.0), (0.0, -1.0)][4 * m // R]
    a = 2 * math.pi * min(m, R - m) / R
    return math.cos(a), math.sin(a) if m <= R - m else -math.sin(a)


def flit(x):
    t = f"{x:.17g}"
    return (t if ("." in t or "e" in t) else t + ".0") + "f"
ROW_LDS = 32 * 1024
# at least this many complex values per wave (rows of short half-rows)
ROW_ELEMS = 512


def row_radices(M):
    return radices(M, big=8, merge=False)


def row_rows(M):
    """Rows per wave: enough for the largest-radix stage to give nearly every
    lane a butterfly; where that count does not fill exactly one round of
    64 butterflies, at least ROW_ELEMS complex values per wave (measured:
    short half-rows such as 54, 108 and 125 points gain 5-24 % in the x
    passes, those whose stage already fills one round, such as 64, 80 and
    128, do not), within 16 rows and ROW_LDS bytes of rows per workgroup."""
    rmax = max(row_radices(M))
    cap = max(1, min(16, ROW_LDS // (4 * M * 8)))
    base = max(1, min(cap, -(-64 * rmax // M)))
    if base * M == 64 * rmax:
        return base
    return max(base, min(cap, -(-ROW_ELEMS // M)))


MAX_COL = 1024
MAX_ROW = 1024


def col_threads(L):
    return 64 if L <= 48 else 128 if L <= 128 else 256 if L <= 256 or L == 512 else 512


def col_lines(L):
    """Lines per column tile: 16 (128-byte row segments) up to 512 points,
    8 above (the tile of 1024 points then takes 64 KB of LDS)."""
    return 16 if L <= 512 else 8


def col_class(L):
    """Length class of a column length: 0 (<= 48), 1 (<= 128), 2 (<= 256),
    3 (256 < L < 512), 4 (512), 5 (512 < L <= 1024)."""
    return 0 if L <= 48 else 1 if L <= 128 else 2 if L <= 256 else 4 if L == 512 else 3 if L < 512 else 5


def col_classes():
    out = []
    cols = smooth5(8, MAX_COL)
    for c in range(6):
        ls = [L for L in cols if col_class(L) == c]
        ts = {(col_threads(L), col_lines(L)) for L in ls}
        assert len(ts) == 1
        t, tx = ts.pop()
        out.append((t, tx, max(ls), ls))
    return out


def main():
    lines = ["// Generated by gen_exact_lengths.py: lengths with compile-time transform",
             "// plans for every 5-smooth size.  Do not edit by hand.",
             "#pragma once", "",
             "// X(L, threads, lines per tile, radices...)",
             "#define MVD_EXACT_COL(X) \\"]
    cols = smooth5(8, MAX_COL)
    for i, L in enumerate(cols):
        end = " \\" if i + 1 < len(cols) else ""
        lines.append(f"  X({L}, {col_threads(L)}, {col_lines(L)}, {', '.join(map(str, radices(L)))}){end}")
    lines += ["", "// X(M, waves per workgroup, rows per wave, radices...)", "#define MVD_EXACT_ROW(X) \\"]
    rows = smooth5(4, MAX_ROW)
    for i, M in enumerate(rows):
        end = " \\" if i + 1 < len(rows) else ""
        rad = row_radices(M)
        rpw = row_rows(M)
        lines.append(f"  X({M}, 4, {rpw}, {', '.join(map(str, rad))}){end}")
    lines.append("")
    # column length classes: the per-length plans of one thread count and
    # length range, for kernels that serve blocks of several lengths
    lines += ["", "// Column length classes: X(class, threads, lines per tile, longest length,",
              "// plans...), each plan ColPlan<L, radices...>.", "#define MVD_COL_CLASSES(X) \\"]
    cls = col_classes()
    for i, (t, tx, lmax, ls) in enumerate(cls):
        end = " \\" if i + 1 < len(cls) else ""
        plans = ", ".join(f"ColPlan<{L}, {', '.join(map(str, radices(L)))}>" for L in ls)
        lines.append(f"  X({i}, {t}, {tx}, {lmax}, {plans}){end}")
    lines += ["", "// X(L, class) for every column length", "#define MVD_COL_CLASS_OF(X) \\"]
    cols = smooth5(8, MAX_COL)
    for i, L in enumerate(cols):
        end = " \\" if i + 1 < len(cols) else ""
        lines.append(f"  X({L}, {col_class(L)}){end}")
    lines.append("")
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "mvd_exact_lengths.h")
    open(path, "w").write("\n".join(lines))
    print(f"{len(cols)} column lengths, {len(rows)} row lengths -> {path}")
    tw = ["// Generated by gen_exact_lengths.py: cos and sin of 2 pi m / R, m < R, for",
          "// the composite radices (FP64 values rounded once to FP32).  Do not edit",
          "// by hand.", "#pragma once", "", "namespace mvdk {", "",
          "template <int R>", "struct SmallTw;", ""]
    for R in COMPOSITE:
        cs = [unit(m, R) for m in range(R)]
        c = ", ".join(flit(x[0]) for x in cs)
        sn = ", ".join(flit(x[1]) for x in cs)
        tw += ["template <>", f"struct SmallTw<{R}> {{", f"  static constexpr float c[{R}] = {{{c}}};",
               f"  static constexpr float s[{R}] = {{{sn}}};", "};", ""]
    tw += ["}  // namespace mvdk", ""]
    path = os.path.join(here, "fft_small_tw.h")
    open(path, "w").write("\n".join(tw))
    print(f"{len(COMPOSITE)} composite radices -> {path}")


if __name__ == "__main__":
    main()
