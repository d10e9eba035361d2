"""LDS line layouts of the transform kernels (host-side checks, no GPU).

The kernels place element x of a buffer of FFT lines at at(x) = x ^ T(x >> B)
with the tables of csrc/lds_swizzle.hpp, and form addresses as a per-thread
base XOR compile-time constants, relying on at() and the digit reversal being
linear over GF(2). These tests re-derive those addresses in Python and check
them against the direct definitions for every table, line length and thread
count the kernels use, and check the pair-unit DCT post/pre-processing
identities numerically against the plain DCT definitions.
"""
import os
import re
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2601_10057_amd", "csrc")
sys.path.insert(0, CSRC)
import gen_lds_swizzle as G  # noqa: E402

pytestmark = pytest.mark.filterwarnings("ignore")


def load_tables():
    txt = open(os.path.join(CSRC, "lds_swizzle.hpp")).read()
    tabs = {}
    for esz, n, cls, cols in re.findall(
            r"struct SwzTab<(\d+), (\d+), (SWZ_\w+)> \{\n  static constexpr int NC = \d+;\n"
            r"  static constexpr int col\[\d+\] = \{([^}]*)\};", txt):
        tabs[(int(esz), int(n), cls)] = [int(v) for v in cols.split(",")]
    return tabs


TABLES = load_tables()


def mapper(esz, n, cls):
    cols = TABLES.get((esz, n, cls), [])
    b = 5 if esz == 8 else 4

    def at(x):
        r = x
        for i, c in enumerate(cols):
            if (x >> (b + i)) & 1:
                r ^= c
        return r
    return at


def test_tables_present_for_every_line_length():
    for esz in (8, 16):
        b = 5 if esz == 8 else 4
        for n in G.SIZES:
            for cls in G.CLASSES:
                if G.buffer_bits(esz, n, cls) > b:
                    assert (esz, n, cls) in TABLES, (esz, n, cls)


@pytest.mark.parametrize("esz", [8, 16])
@pytest.mark.parametrize("cls", G.CLASSES)
def test_map_is_a_permutation_inside_aligned_groups(esz, cls):
    b = 5 if esz == 8 else 4
    for n in G.SIZES:
        at = mapper(esz, n, cls)
        size = 1 << G.buffer_bits(esz, n, cls)
        y = np.array([at(x) for x in range(size)])
        assert sorted(y) == list(range(size))
        assert np.all((y >> b) == (np.arange(size) >> b))


def line_slots(n, nthr, radix, at):
    """Base-XOR-constant slots of LineSlots (fft.hpp) for every thread."""
    def g(k):
        return at(G.digit_rev(k, n, radix))
    out = {}
    lpt = n // nthr if n >= nthr else 1
    upt = n // 2 // nthr if n // 2 >= nthr else 1
    for tid in range(nthr):
        t = tid
        nat0 = at(t)
        mak0 = at(t >> 1) ^ (at(n - 1) if t & 1 else 0)
        bin0 = g(t)
        out0 = g(t >> 1) ^ (at(n - 1) if t & 1 else 0)
        natm0 = at(n - 1) ^ at((t - 1) & (n - 1))
        binm0 = at(n - 1) ^ g((t - 1) & (n - 1))
        for q in range(lpt):
            i = t + q * nthr
            if i >= n:
                continue
            out[("nat", tid, q)] = (nat0 ^ at(q * nthr), at(i))
            out[("mak", tid, q)] = (mak0 ^ at(q * (nthr // 2)), at(G.makhoul_slot(i, n)))
            out[("bin", tid, q)] = (bin0 ^ g(q * nthr), g(i))
            out[("out", tid, q)] = (out0 ^ g(q * (nthr // 2)), g(G.makhoul_slot(i, n)))
        for q in range(upt):
            u = t + q * nthr
            if u >= n // 2:
                continue
            mirror = n - u if u else n // 2
            if t == 0:
                c_nat = at(n // 2) if q == 0 else at(n - 1) ^ at((q * nthr - 1) & (n - 1))
                c_bin = g(n // 2) if q == 0 else at(n - 1) ^ g((q * nthr - 1) & (n - 1))
            else:
                c_nat = natm0 ^ at(q * nthr)
                c_bin = binm0 ^ g(q * nthr)
            out[("natm", tid, q)] = (c_nat, at(mirror))
            out[("binm", tid, q)] = (c_bin, g(mirror))
    return out


@pytest.mark.parametrize("esz", [8, 16])
def test_line_slots_match_direct_definitions(esz):
    radix = G.fft_radix(esz)
    for n in G.SIZES:
        for cls, nthrs, rad in (
                ("SWZ_LINE", {G.line_threads(n), G.one_line_threads(esz, n)}, radix),
                ("SWZ_GRAM", {G.gram_threads(esz, n)}, G.gram_radix(esz, n)),
                ("SWZ_ROW", {G.row_dct_threads(n, 0), G.row_dct_threads(n, 1),
                             G.row_idct_threads(esz, n)}, radix)):
            at = mapper(esz, n, cls)
            for nthr in nthrs:
                for key, (fast, direct) in line_slots(n, nthr, rad, at).items():
                    assert fast == direct, (esz, n, cls, nthr, key)


@pytest.mark.parametrize("esz", [8, 16])
def test_row_dct_post_slots(esz):
    """Slots of bins 2 sp, 2 sp + 1 and their mirrors in the row DCT, where
    HALVES adjacent lanes share column pair sp = t / HALVES + it NTHR / HALVES."""
    radix = G.fft_radix(esz)
    for n in G.SIZES:
        at = mapper(esz, n, "SWZ_ROW")

        def g(k):
            return at(G.digit_rev(k, n, radix))
        for v in (0, 1):
            nthr = G.row_dct_threads(n, v)
            halves = 2 if G.p1_rows_v(esz, n, v) >= 2 else 1
            spl = nthr // halves
            spt_n = n // 2 // spl if n // 2 >= spl else 1
            for tid in range(nthr):
                spt = tid // halves
                g2 = g(2 * spt)
                g2m = at(n - 1) ^ g(1) ^ g((2 * spt - 2) & (n - 1))
                for it in range(spt_n):
                    sp = spt + it * spl
                    if sp >= n // 2:
                        continue
                    c0 = 0 if it == 0 else at(n - 1) ^ g(1) ^ g((2 * it * spl - 2) & (n - 1))
                    pk0 = g2 ^ g(2 * it * spl)
                    pk1 = pk0 ^ g(1)
                    pm1 = pk0 ^ at(n - 1)
                    pm0 = c0 if spt == 0 else g2m ^ g(2 * it * spl)
                    assert pk0 == g(2 * sp) and pk1 == g(2 * sp + 1)
                    assert pm0 == g((n - 2 * sp) % n) and pm1 == g(n - 2 * sp - 1)


@pytest.mark.parametrize("esz", [8, 16])
def test_fft_stage_slots(esz):
    """Butterfly slots at(e0(tid)) ^ at(e0(it NTHR)) ^ at(r S) equal at(e0 + r S),
    and every stage touches each element of the buffer exactly once."""
    radix = G.fft_radix(esz)
    for n in G.SIZES:
        cases = [("SWZ_LINE", 1, nt, radix) for nt in {G.line_threads(n), G.one_line_threads(esz, n)}]
        cases.append(("SWZ_GRAM", 1, G.gram_threads(esz, n), G.gram_radix(esz, n)))
        for v in (0, 1):
            cases.append(("SWZ_ROW", G.p1_rows_v(esz, n, v) * G.p1_pairs_v(esz, n, v),
                          G.row_dct_threads(n, v), radix))
        # row inverse over a band of rows
        cases.append(("SWZ_ROW", G.row_idct_rows(esz, n), G.row_idct_threads(esz, n), radix))
        for cls, nl, nthr, rad in cases:
            at = mapper(esz, n, cls)
            length = n
            for r in G.plan(n, rad):
                s = length // r
                tot = (n // r) * nl
                ls, lr = s.bit_length() - 1, r.bit_length() - 1
                iters = tot // nthr if tot >= nthr else 1

                def first(b):
                    return (b & (s - 1)) | ((b >> ls) << (ls + lr))
                seen = []
                for tid in range(min(nthr, tot)):
                    base = at(first(tid))
                    for it in range(iters):
                        e = base ^ at(first(it * nthr))
                        b = tid + it * nthr
                        line, jb = divmod(b, n // r)
                        blk, m = divmod(jb, s)
                        e0 = line * n + blk * length + m
                        for q in range(r):
                            assert e ^ at(q * s) == at(e0 + q * s)
                            seen.append(e ^ at(q * s))
                assert sorted(seen) == list(range(n * nl)), (esz, n, cls, r)
                length //= r


def dct2_ortho(x):
    n = len(x)
    k = np.arange(n)[:, None]
    i = np.arange(n)[None, :]
    c = np.cos(np.pi * k * (2 * i + 1) / (2 * n)) * np.sqrt(2.0 / n)
    c[0] *= np.sqrt(0.5)
    return c @ x


@pytest.mark.parametrize("n", [16, 64, 256])
def test_pair_unit_dct_identities(n):
    """dct2_pair / dct3_pair (fft.hpp) against the orthonormal DCT-II / DCT-III."""
    rng = np.random.default_rng(n)
    a, b = rng.standard_normal(n), rng.standard_normal(n)
    order = [G.makhoul_slot(i, n) for i in range(n)]
    v = np.empty(n, complex)
    v[order] = a + 1j * b                       # Makhoul reordering, z = v_a + i v_b
    Z = np.fft.fft(v)
    w = np.exp(-1j * np.pi * np.arange(n) / (2 * n))
    s1, s0 = 0.5 * np.sqrt(2.0 / n), 0.5 * np.sqrt(1.0 / n)
    A, B = np.zeros(n), np.zeros(n)
    for u in range(n // 2):
        z, zm = Z[u], Z[n - u if u else n // 2]
        v1 = complex(z.real + zm.real, z.imag - zm.imag)
        v2 = complex(z.imag + zm.imag, zm.real - z.real)
        if u:
            p, r = w[u] * v1, w[u] * v2
            A[u], B[u], A[n - u], B[n - u] = s1 * p.real, s1 * r.real, -s1 * p.imag, -s1 * r.imag
        else:
            A[0], B[0] = s0 * 2 * Z[0].real, s0 * 2 * Z[0].imag
            zz = Z[n // 2]
            q1 = w[n // 2] * complex(2 * zz.real, 0)
            q2 = w[n // 2] * complex(2 * zz.imag, 0)
            A[n // 2], B[n // 2] = s1 * q1.real, s1 * q2.real
    assert np.allclose(A, dct2_ortho(a), atol=1e-12)
    assert np.allclose(B, dct2_ortho(b), atol=1e-12)
    # inverse: build the FFT input from the coefficients, pair by pair
    g0, g1 = np.sqrt(n) / n, np.sqrt(0.5 * n) / n
    X = np.zeros(n, complex)
    for u in range(n // 2):
        if u:
            x1, x2, x1m, x2m = A[u] * g1, B[u] * g1, A[n - u] * g1, B[n - u] * g1
            cr, ci = w[u].real, -w[u].imag
            v1r, v1i = cr * x1 + ci * x1m, ci * x1 - cr * x1m
            v2r, v2i = cr * x2 + ci * x2m, ci * x2 - cr * x2m
            X[u] = complex(v1r - v2i, -(v1i + v2r))
            X[n - u] = complex(v1r + v2i, v1i - v2r)
        else:
            X[0] = complex(A[0] * g0, -(B[0] * g0))
            x1, x2 = A[n // 2] * g1, B[n // 2] * g1
            cr, ci = w[n // 2].real, -w[n // 2].imag
            v1r, v1i = (cr + ci) * x1, (ci - cr) * x1
            v2r, v2i = (cr + ci) * x2, (ci - cr) * x2
            X[n // 2] = complex(v1r - v2i, -(v1i + v2r))
    y = np.fft.fft(X)
    assert np.allclose(y.real[order], a, atol=1e-12)
    assert np.allclose(-y.imag[order], b, atol=1e-12)
