"""Choose the LDS layouts of the transform kernels' lines and write lds_swizzle.hpp.

Element x of a buffer of FFT lines lives in LDS at x ^ T(x >> B), where T is a
linear map over GF(2) from the bits above B to the low B bits, with B = 5 for
8-byte (FP32 complex) and B = 4 for 16-byte (FP64 complex) elements. The map
only permutes elements inside aligned groups of 2^B, and being linear it lets
a kernel form every address as a per-thread base XOR a compile-time constant.

T is chosen per element size, line length and kernel class by hill climbing on
a model of the LDS: 64 banks of 4 bytes; an instruction of a 64-lane wave is
served in groups of 256 / (element size) lanes; a group takes as many cycles
as the largest number of distinct dwords that fall into one bank. The cost of
a layout is the modelled number of cycles over every line access of the class
(FFT stage reads and writes, the Makhoul-ordered loads, the post-processing
reads in digit-reversed order, the natural-order writes of the inverse). The
index rules below follow the kernels in fft.hpp and step_kernels.hpp; a
change there needs a change here and a new header.

Usage: python gen_lds_swizzle.py  (rewrites lds_swizzle.hpp next to this file)
"""
from __future__ import annotations

import math
import os
import random
import sys
from multiprocessing import Pool

import numpy as np

CLASSES = ("SWZ_ROW", "SWZ_LINE", "SWZ_GRAM")
SIZES = [1 << k for k in range(4, 14)]          # line lengths 16 .. 8192


# ---- launch shapes (mirror step_kernels.hpp) --------------------------------
def clamp_threads(t):
    return 64 if t < 64 else (1024 if t > 1024 else t)


def line_threads(n):
    return clamp_threads(n // 4)


def one_line_threads(esz, n):
    return clamp_threads(n // (16 if esz == 8 else 8))


def gram_threads(esz, n):
    return clamp_threads(n // (16 if esz == 8 and n >= 8192 else 8))


def fft_radix(esz):
    return 16 if esz == 8 else 8


def gram_radix(esz, n):
    q = n // gram_threads(esz, n)
    return 8 if q >= 8 else (4 if q >= 4 else 2)


def lds_line_budget(esz, n):
    return (136 * 1024) // (n * esz)


def p1_rows(esz, n):
    want = 32 // (2 * (esz // 2))
    fit = lds_line_budget(esz, n)
    return want if fit >= want else (2 if fit >= 2 else 1)


def p1_pairs(esz, n):
    per = lds_line_budget(esz, n) // p1_rows(esz, n)
    return 4 if per >= 4 else (2 if per >= 2 else 1)


def p1_rows_v(esz, n, v):
    r = p1_rows(esz, n) >> v
    return r if r > 0 else 1


def p1_pairs_v(esz, n, v):
    lines0 = p1_rows(esz, n) * p1_pairs(esz, n)
    rows = p1_rows_v(esz, n, v)
    lines = max(lines0 >> v, rows)
    per = lines // rows
    return 4 if per >= 4 else (2 if per >= 2 else 1)


def row_dct_threads(n, v):
    return line_threads(n)


def row_idct_rows(esz, n):
    """Rows per workgroup of the band row inverse (launch variant 0)."""
    return max(p1_rows(esz, n) // 2, 1)


def row_idct_threads(esz, n):
    bf = row_idct_rows(esz, n) * n // fft_radix(esz)
    return clamp_threads(bf) if bf < line_threads(n) else line_threads(n)


# ---- FFT index rules (mirror fft.hpp) ----------------------------------------
def ilog2(n):
    return n.bit_length() - 1


def plan(n, radix):
    lg, lr = ilog2(n), ilog2(radix)
    rem = lg % lr
    rs = [radix if rem == 0 else 1 << rem]
    m = n // rs[0]
    while m > 1:
        rs.append(radix)
        m //= radix
    return rs


def digit_rev(k, n, radix):
    span, p = n, 0
    for r in plan(n, radix):
        span //= r
        p += (k % r) * span
        k //= r
    return p


def makhoul_slot(i, n):
    return n - 1 - (i >> 1) if i & 1 else i >> 1


# ---- access recording ---------------------------------------------------------
class Rec:
    """Collects the element positions of each lane group of each LDS access."""

    def __init__(self, esz):
        self.g = 256 // esz
        self.rows = []

    def wave(self, pos):
        for g0 in range(0, 64, self.g):
            grp = [p for p in pos[g0:g0 + self.g] if p is not None]
            if grp:
                self.rows.append(grp + [-1] * (self.g - len(grp)))


def lanes(nthr):
    for w0 in range(0, nthr, 64):
        yield range(w0, min(w0 + 64, nthr))


def rec_fft(rec, n, nl, nthr, radix):
    length = n
    for r in plan(n, radix):
        s = length // r
        nb = n // r
        tot = nb * nl
        for w in lanes(nthr):
            for b0 in range(0, tot, nthr):
                e0 = []
                for t in w:
                    b = b0 + t
                    if b >= tot:
                        e0.append(None)
                        continue
                    line, jb = divmod(b, nb)
                    blk, m = divmod(jb, s)
                    e0.append(line * n + blk * length + m)
                for q in range(r):
                    pos = [None if e is None else e + q * s for e in e0]
                    rec.wave(pos)      # read
                    rec.wave(pos)      # write
        length //= r


def rec_makhoul(rec, n, nthr, line=0):
    for w in lanes(nthr):
        for i0 in range(0, n, nthr):
            rec.wave([line * n + makhoul_slot(i0 + t, n) if i0 + t < n else None for t in w])


def rec_pair_post(rec, n, nthr, radix):
    for w in lanes(nthr):
        for u0 in range(0, n // 2, nthr):
            us = [u0 + t if u0 + t < n // 2 else None for t in w]
            rec.wave([None if u is None else digit_rev(u, n, radix) for u in us])
            rec.wave([None if u is None else digit_rev(n - u if u else n // 2, n, radix) for u in us])


def rec_pair_natural(rec, n, nthr, line=0):
    for w in lanes(nthr):
        for u0 in range(0, n // 2, nthr):
            us = [u0 + t if u0 + t < n // 2 else None for t in w]
            rec.wave([None if u is None else line * n + u for u in us])
            rec.wave([None if u is None else line * n + (n - u if u else n // 2) for u in us])


def rec_final(rec, n, nthr, radix, line=0):
    for w in lanes(nthr):
        for i0 in range(0, n, nthr):
            rec.wave([line * n + digit_rev(makhoul_slot(i0 + t, n), n, radix) if i0 + t < n else None
                      for t in w])


def rec_band_inverse(rec, n, nthr, radix, rows):
    """Row inverse over a band: strip pieces stored by column pair, the in-place
    DCT-III pre-processing, the batched FFT and the outputs, row by row."""
    for w in lanes(nthr):
        for s0 in range(0, n // 2, nthr):
            sts = [s0 + t if s0 + t < n // 2 else None for t in w]
            for r in range(rows):
                for kk in (0, 1):
                    rec.wave([None if st is None else r * n + 2 * st + kk for st in sts])
    for r in range(rows):
        rec_pair_natural(rec, n, nthr, r)      # reads
        rec_pair_natural(rec, n, nthr, r)      # writes
    rec_fft(rec, n, rows, nthr, radix)
    for r in range(rows):
        rec_final(rec, n, nthr, radix, r)


def patterns(esz, n, cls):
    """Position arrays (one row per lane group) of every access of the class."""
    rec = Rec(esz)
    radix = fft_radix(esz)
    if cls == "SWZ_ROW":
        for v in (0, 1):
            nthr = row_dct_threads(n, v)
            nl = p1_rows_v(esz, n, v) * p1_pairs_v(esz, n, v)
            for ln in range(nl):
                rec_makhoul(rec, n, nthr, ln)
            rec_fft(rec, n, nl, nthr, radix)
            rows = p1_rows_v(esz, n, v)
            npairs = nl // rows
            halves = 2 if rows >= 2 else 1
            rh = rows // halves
            spl = nthr // halves
            for w in lanes(nthr):
                for s0 in range(0, n // 2, spl):
                    sps = [s0 + t // halves if s0 + t // halves < n // 2 else None for t in w]
                    hs = [t % halves for t in w]
                    for l in range(npairs):
                        for q in range(rh):
                            lns = [(h * rh + q) * npairs + l for h in hs]
                            for kk in (0, 1):
                                ks = [None if sp is None else 2 * sp + kk for sp in sps]
                                rec.wave([None if k is None else ln * n + digit_rev(k, n, radix)
                                          for k, ln in zip(ks, lns)])
                                rec.wave([None if k is None else ln * n + digit_rev((n - k) % n, n, radix)
                                          for k, ln in zip(ks, lns)])
        rec_band_inverse(rec, n, row_idct_threads(esz, n), radix, row_idct_rows(esz, n))
    elif cls == "SWZ_LINE":
        for nthr in sorted({line_threads(n), one_line_threads(esz, n)}):
            # column solve
            rec_makhoul(rec, n, nthr)
            rec_fft(rec, n, 1, nthr, radix)
            rec_pair_post(rec, n, nthr, radix)
            rec_pair_natural(rec, n, nthr)
            rec_fft(rec, n, 1, nthr, radix)
            rec_final(rec, n, nthr, radix)
        # row inverse, one row with one butterfly per thread
        nthr = one_line_threads(esz, n)
        rec_pair_natural(rec, n, nthr)
        rec_fft(rec, n, 1, nthr, radix)
        rec_final(rec, n, nthr, radix)
        # row DCT of a single field
        nthr = line_threads(n)
        rec_makhoul(rec, n, nthr)
        rec_fft(rec, n, 1, nthr, radix)
        rec_pair_post(rec, n, nthr, radix)
    else:
        nthr = gram_threads(esz, n)
        gr = gram_radix(esz, n)
        rec_makhoul(rec, n, nthr)
        rec_fft(rec, n, 1, nthr, gr)
        rec_pair_post(rec, n, nthr, gr)
    return np.array(rec.rows, dtype=np.int64)


def buffer_bits(esz, n, cls):
    if cls == "SWZ_ROW":
        nl = max(p1_rows_v(esz, n, v) * p1_pairs_v(esz, n, v) for v in (0, 1))
        return ilog2(n * nl)
    return ilog2(n)


# ---- cost and search ----------------------------------------------------------
def table(cols, nb):
    tab = np.zeros(1 << len(cols), dtype=np.int64)
    for h in range(1 << len(cols)):
        v = 0
        for b, c in enumerate(cols):
            if (h >> b) & 1:
                v ^= c
        tab[h] = v
    return tab


def cost(P, cols, nb):
    valid = P >= 0
    x = np.where(valid, P, 0)
    hi = (x >> nb) & ((1 << len(cols)) - 1)
    y = x ^ table(cols, nb)[hi]
    key = y & ((1 << nb) - 1)
    width = 1 << nb
    flat = np.where(valid, np.arange(P.shape[0])[:, None] * width + key, P.shape[0] * width)
    cnt = np.bincount(flat.ravel(), minlength=P.shape[0] * width + 1)[:-1]
    return int(cnt.reshape(P.shape[0], width).max(axis=1).sum())


def climb(P, nc, nb, seed, sweeps=8):
    rng = random.Random(seed)
    cols = [rng.randrange(1 << nb) for _ in range(nc)]
    best = cost(P, cols, nb)
    for _ in range(sweeps):
        improved = False
        for b in rng.sample(range(nc), nc):
            for v in range(1 << nb):
                if v == cols[b]:
                    continue
                old, cols[b] = cols[b], v
                c = cost(P, cols, nb)
                if c < best:
                    best, improved = c, True
                else:
                    cols[b] = old
        if not improved:
            break
    return best, cols


def solve(job):
    esz, n, cls = job
    nb = 5 if esz == 8 else 4
    nc = max(0, buffer_bits(esz, n, cls) - nb)
    P = patterns(esz, n, cls)
    base = cost(P, [0] * nc, nb) if nc else cost(P, [], nb)
    if nc == 0:
        return job, [], base, base, P.shape[0]
    best = None
    for seed in range(6):
        c, cols = climb(P, nc, nb, 1000 * n + 10 * esz + seed)
        if best is None or c < best[0]:
            best = (c, cols)
    return job, best[1], best[0], base, P.shape[0]


def main():
    jobs = [(esz, n, cls) for esz in (8, 16) for n in SIZES for cls in CLASSES]
    with Pool(min(8, os.cpu_count() or 1)) as pool:
        results = pool.map(solve, jobs)
    out = [
        "// Generated by gen_lds_swizzle.py; do not edit by hand.",
        "//",
        "// XOR layouts of the LDS lines of the transform kernels: element x of a",
        "// buffer of lines lives at x ^ T(x >> B), T(h) = XOR of col[b] over the set",
        "// bits b of h (B = 5 for 8-byte, 4 for 16-byte elements). Per table: the",
        "// modelled LDS cycles per lane group over the class's accesses, with this",
        "// layout and with the plain layout (ideal 1.0).",
        "#pragma once",
        "",
        "namespace ccm {",
        "",
        "enum SwzClass { SWZ_ROW = 0, SWZ_LINE = 1, SWZ_GRAM = 2 };",
        "",
        "template <int ESZ, int N, int CLS> struct SwzTab {",
        "  static constexpr int NC = 0;",
        "  static constexpr int col[1] = {0};",
        "};",
        "",
    ]
    for (esz, n, cls), cols, c, base, groups in results:
        if not cols:
            continue
        out.append(f"// {esz}-byte elements, N = {n}, {cls}: {c / groups:.3f} cycles/group "
                   f"(plain {base / groups:.3f})")
        out.append(f"template <> struct SwzTab<{esz}, {n}, {cls}> {{")
        out.append(f"  static constexpr int NC = {len(cols)};")
        out.append(f"  static constexpr int col[{len(cols)}] = {{{', '.join(str(v) for v in cols)}}};")
        out.append("};")
    out += ["", "}  // namespace ccm", ""]
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lds_swizzle.hpp")
    with open(path, "w") as f:
        f.write("\n".join(out))
    print(f"wrote {path}")


if __name__ == "__main__":
    sys.exit(main())
