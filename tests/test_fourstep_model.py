"""The factored (four-step) DCT of the DCT-as-GEMM variant, as a CPU model
(gemm_fourstep.hpp, gemm_mfma.hpp, upload_fs_matrices in ccmsav_runtime.hip):
the four matrices and two twiddle tables built by the same formulas as the
library, the products as exact matrix products, and every flat index of the
operand loads and epilogues as the kernels form it. Work buffers start as
NaN, so an element the model never writes shows up.

- Forward (DCT-II) and inverse (DCT-III) along rows and along columns match
  scipy's orthonormal DCT to 1e-13 for N1 x N2 = 4 x 8, 8 x 4, 4 x 4, 8 x 8
  with several lines and fields (the index rules do not depend on the sizes
  beyond their being powers of two).
- The forward matrices alone give the DFT of the reordered line: the
  Makhoul identity the derivation rests on.
"""
import numpy as np
import pytest
from scipy.fft import dct, fft


def ex(num, den):
    """exp(-i pi num / den) as (cos, sin), num reduced mod 2 den (as the library)."""
    a = np.pi * (np.asarray(num) % (2 * den)) / den
    return np.cos(a), -np.sin(a)


def build(n1, n2):
    """d1, d2 (forward), d1i, d2i (inverse), twf, twi as upload_fs_matrices."""
    n = n1 * n2
    d1 = np.zeros((2 * n1, n1))
    d1i = np.zeros((2 * n1, 2 * n1))
    d2 = np.zeros((n2, 2 * n2))
    d2i = np.zeros((n2, 2 * n2))
    up, down = np.sqrt(0.5 * n), np.sqrt(2.0 / n)
    for k in range(n1):
        for j in range(n1):
            c, s = ex(2 * j * k, n1)
            d1[2 * k, j], d1[2 * k + 1, j] = c, s
            c, s = ex(j * (4 * k + 1), 2 * n1)
            c, s = c * up, s * up
            d1i[2 * k, j], d1i[2 * k, n1 + j] = c, -s
            d1i[2 * k + 1, j], d1i[2 * k + 1, n1 + j] = s, c
    for k in range(n2):
        for j in range(n2):
            c, s = ex(k * (4 * j + 1), 2 * n2)
            d2[k, j], d2[k, n2 + j] = down * c, -down * s
            c, s = ex(2 * j * k, n2)
            d2i[k, j], d2i[k, n2 + j] = c / n, -s / n
    twf = np.zeros((n, 2))
    twi = np.zeros((n, 2))
    for k1 in range(n1):
        for j in range(n2):
            twf[k1 * n2 + j] = ex(k1 * (4 * j + 1), 2 * n)
            twi[k1 * n2 + j] = ex(j * (4 * k1 + 1), 2 * n)
    return d1, d2, d1i, d2i, twf, twi


def src(j, n):
    return np.where(j < n // 2, 2 * j, 2 * (n - 1 - j) + 1)


def place(m, n):
    return np.where(m < n // 2, 2 * m, 2 * (n - 1 - m) + 1)


def load(xl, x, z, k, m, f):
    """Step 1's data operand element (k, m) of batch entry z (fs_load)."""
    l1, l2, lx = f
    ln = l1 + l2
    n = 1 << ln
    n1m = (1 << l1) - 1
    if xl == "makhoul_rows":
        return x[(z << ln) + src((k << l2) + m, n)]
    if xl == "makhoul_cols":
        return x[(src((k << l2) + z, n) << lx) + m]
    j = ((k & n1m) << l2) + (m if xl == "z_rows" else z)
    im = k > n1m
    base = (z << ln) if xl == "z_rows" else m
    stride = 1 if xl == "z_rows" else (1 << lx)
    re_v = np.where(j == 0, x[base] * np.sqrt(2.0), x[base + j * stride])
    im_v = np.where(j == 0, 0.0, x[base + np.where(j == 0, 0, n - j) * stride])
    return np.where(im, im_v, re_v)


def product(mode, d, x, M, N, K, ldx, sx, batch, xl=None, f=None):
    """C[z, n, m] of the row or column mode (gemm_mfma.hpp)."""
    out = np.zeros((batch, N, M))
    kk, mm = np.meshgrid(np.arange(K), np.arange(M), indexing="ij")
    for z in range(batch):
        if mode == "row":
            X = np.stack([x[z * sx + n * ldx: z * sx + n * ldx + K] for n in range(N)])
            out[z] = X @ d.reshape(-1)[:M * K].reshape(M, K).T
        else:
            X = load(xl, x, z, kk, mm, f) if xl else x[z * sx + kk * ldx + mm]
            out[z] = d.reshape(-1)[:N * K].reshape(N, K) @ X
    return out


def epilogue(epi, C, c, ldc, sc, f, tw):
    """fs_epilogue over every element pair of C."""
    l1, l2, lx = f
    ln = l1 + l2
    nn = 1 << ln
    n1m = (1 << l1) - 1
    B, N, M = C.shape
    swap = epi in ("post_rows", "ipost_rows")
    z, n, m = np.meshgrid(np.arange(B), np.arange(N), np.arange(M), indexing="ij")
    sel = (m % 2 == 0) if swap else (n % 2 == 0)
    z, n, m = z[sel], n[sel], m[sel]
    x0 = C[z, n, m]
    x1 = C[z, n, m + 1] if swap else C[z, n + 1, m]
    if epi in ("tw_m", "tw_z"):
        w = tw[((n >> 1) << l2) + (m if epi == "tw_m" else z)]
        c[z * sc + n * ldc + m] = x0 * w[:, 0] - x1 * w[:, 1]
        c[z * sc + (n + 1) * ldc + m] = x0 * w[:, 1] + x1 * w[:, 0]
    elif epi == "post_rows":
        k = (n & n1m) + (m << l1)
        y = (n >> l1) << ln
        c[y + k] = np.where(k == 0, x0 * np.sqrt(0.5), x0)
        c[y + k + (1 << l1)] = x1
    elif epi == "post_cols":
        k = (z & n1m) + (n << l1)
        y = ((z >> l1) << (ln + lx)) + m
        c[y + (k << lx)] = np.where(k == 0, x0 * np.sqrt(0.5), x0)
        c[y + ((k + (1 << l1)) << lx)] = x1
    elif epi == "ipost_rows":
        xo = (n >> l1) << ln
        b1 = n & n1m
        c[xo + place(b1 + (m << l1), nn)] = x0
        c[xo + place(b1 + ((m + 1) << l1), nn)] = x1
    else:
        xo = ((z >> l1) << (ln + lx)) + m
        b1 = z & n1m
        c[xo + (place(b1 + (n << l1), nn) << lx)] = x0
        c[xo + (place(b1 + ((n + 1) << l1), nn) << lx)] = x1


def rows(x, lines, l1, l2, inverse):
    d1, d2, d1i, d2i, twf, twi = build(1 << l1, 1 << l2)
    n1, n2 = 1 << l1, 1 << l2
    n = n1 * n2
    f = (l1, l2, 0)
    t = np.full(2 * lines * n, np.nan)
    y = np.full(lines * n, np.nan)
    if not inverse:
        C = product("col", d1, x, n2, 2 * n1, n1, 0, 0, lines, "makhoul_rows", f)
        epilogue("tw_m", C, t, n2, 2 * n, f, twf)
        epilogue("post_rows", product("row", d2, t, n2, lines * n1, 2 * n2, 2 * n2, 0, 1),
                 y, 0, 0, f, None)
    else:
        C = product("col", d1i, x, n2, 2 * n1, 2 * n1, 0, 0, lines, "z_rows", f)
        epilogue("tw_m", C, t, n2, 2 * n, f, twi)
        epilogue("ipost_rows", product("row", d2i, t, n2, lines * n1, 2 * n2, 2 * n2, 0, 1),
                 y, 0, 0, f, None)
    return y


def cols(x, fields, l1, l2, lx, inverse):
    d1, d2, d1i, d2i, twf, twi = build(1 << l1, 1 << l2)
    n1, n2, nx = 1 << l1, 1 << l2, 1 << lx
    cells = n1 * n2 * nx
    f = (l1, l2, lx)
    t = np.full(2 * fields * cells, np.nan)
    y = np.full(fields * cells, np.nan)
    for fl in range(fields):
        tv = t[2 * fl * cells:]
        xf = x[fl * cells:]
        if not inverse:
            C = product("col", d1, xf, nx, 2 * n1, n1, 0, 0, n2, "makhoul_cols", f)
        else:
            C = product("col", d1i, xf, nx, 2 * n1, 2 * n1, 0, 0, n2, "z_cols", f)
        epilogue("tw_z", C, tv, n2 * nx, nx, f, twi if inverse else twf)
    sv = 2 * n2 * nx
    C = product("col", d2i if inverse else d2, t, nx, n2, 2 * n2, nx, sv, fields * n1)
    epilogue("ipost_cols" if inverse else "post_cols", C, y, 0, 0, f, None)
    return y


SHAPES = [(2, 3, 2, 3), (3, 2, 3, 2), (2, 2, 4, 1), (3, 3, 2, 2)]


@pytest.mark.parametrize("l1,l2,lx,fields", SHAPES)
def test_rows_forward_and_inverse_match_the_orthonormal_dct(l1, l2, lx, fields):
    n = 1 << (l1 + l2)
    lines = 5 * fields
    rng = np.random.default_rng(l1 * 10 + l2)
    x = rng.standard_normal(lines * n)
    ref = dct(x.reshape(lines, n), type=2, norm="ortho", axis=1).ravel()
    assert np.abs(rows(x, lines, l1, l2, False) - ref).max() < 1e-13
    assert np.abs(rows(ref, lines, l1, l2, True) - x).max() < 1e-13


@pytest.mark.parametrize("l1,l2,lx,fields", SHAPES)
def test_columns_forward_and_inverse_match_the_orthonormal_dct(l1, l2, lx, fields):
    n, nx = 1 << (l1 + l2), 1 << lx
    rng = np.random.default_rng(100 + l1 * 10 + l2)
    x = rng.standard_normal(fields * n * nx)
    ref = dct(x.reshape(fields, n, nx), type=2, norm="ortho", axis=1).ravel()
    assert np.abs(cols(x, fields, l1, l2, lx, False) - ref).max() < 1e-13
    assert np.abs(cols(ref, fields, l1, l2, lx, True) - x).max() < 1e-13


def test_forward_matrices_give_the_dft_of_the_reordered_line():
    # Without the turn and scale folded into d2: P = d1 v, T = P W_N^(n2 k1),
    # V[k1 + N1 k2] = sum_n2 W_N2^(n2 k2) T[k1][n2] is the DFT of v.
    n1, n2 = 4, 8
    n = n1 * n2
    rng = np.random.default_rng(7)
    x = rng.standard_normal(n)
    v = x[src(np.arange(n), n)]
    d1 = build(n1, n2)[0]
    P = d1 @ v.reshape(n1, n2)
    Pc = P[0::2] + 1j * P[1::2]
    k1 = np.arange(n1)[:, None]
    j = np.arange(n2)[None, :]
    T = Pc * np.exp(-2j * np.pi * j * k1 / n)
    V = np.fft.fft(T, axis=1)                      # over n2, output k2
    got = np.empty(n, complex)
    got[(k1 + n1 * np.arange(n2)[None, :]).ravel()] = V.ravel()
    assert np.abs(got - fft(v)).max() < 1e-12
    # and the DCT-II is the turned real part
    k = np.arange(n)
    s = np.where(k == 0, np.sqrt(1.0 / n), np.sqrt(2.0 / n))
    y = s * (np.exp(-1j * np.pi * k / (2 * n)) * fft(v)).real
    assert np.abs(y - dct(x, type=2, norm="ortho")).max() < 1e-12
