// The factored ("four-step") form of the DCT-as-GEMM transforms, for lines of
// N = N1 N2 points, with W_M = exp(-2 pi i / M) and theta_k = pi k / 2N.
//
// Forward (the orthonormal DCT-II of App. C, by FFT means): with the Makhoul
// reordering v of a line x (v_n = x_2n, v_{N-1-n} = x_{2n+1}) and V its DFT,
// y_k = s_k Re(exp(-i theta_k) V_k), s_0 = sqrt(1/N), s_k = sqrt(2/N). The
// DFT of length N1 N2 splits as
//   V[k1 + N1 k2] = sum_n2 W_N2^(n2 k2) W_N^(n2 k1) sum_n1 W_N1^(n1 k1) v[N2 n1 + n2],
// and exp(-i theta_k) = exp(-i pi k1 / 2N) exp(-i pi k2 / 2 N2). So
//   1. P[k1][n2] = sum_n1 W_N1^(n1 k1) v[N2 n1 + n2]          (complex, 2 N1 x N1)
//   2. T = P exp(-i pi k1 (4 n2 + 1) / 2N)                     (twiddle table)
//   3. y[k1 + N1 k2] = Re sum_n2 sqrt(2/N) exp(-i pi k2 (4 n2 + 1) / 2 N2) T[k1][n2]
//      (real outputs, N2 x 2 N2), and y_0 / sqrt 2.
// Inverse (the DCT-III): with w_k = y_k / s_k and w_N = 0, the line is
// x_2n = v_n, x_{2n+1} = v_{N-1-n} for v = Re(DFT(U)) / N,
// U_k = exp(-i theta_k) (w_k + i w_{N-k}). With k = N2 a1 + a2 and
// n = b1 + N1 b2 the turn splits as exp(-i pi a1 / 2 N1) exp(-i pi a2 / 2N):
//   0. Z = y + i (y reversed), Re Z_0 = sqrt 2 y_0, Im Z_0 = 0
//   1. P[b1][a2] = sum_a1 sqrt(N/2) exp(-i pi a1 (4 b1 + 1) / 2 N1) Z[N2 a1 + a2]
//                                                              (complex, 2 N1 x 2 N1)
//   2. T = P exp(-i pi a2 (4 b1 + 1) / 2N)                     (twiddle table)
//   3. v[b1 + N1 b2] = Re sum_a2 W_N2^(a2 b2) T[b1][a2] / N     (real outputs, N2 x 2 N2)
// Steps 1 and 3 are products on the matrix cores (gemm_mfma.hpp) with real
// and imaginary parts stacked along the product dimensions; step 2 and the
// placement of step 3's outputs run in their epilogues. The output rows of
// both complex-output matrices interleave real and imaginary parts (row
// 2 k + re/im), so that both parts of one value land in one lane's
// accumulator (consecutive MFMA rows). The reordering (forward) and step 0
// (inverse) run in step 1's operand loader.
//
// Layouts (FP32) per line (rows: contiguous lines of length N) and per field
// (columns: the lines run along y, nx columns side by side, x contiguous):
//   v  reordered line, read as [n1][n2]        rows [n]          cols [n][x]
//   T  after step 2, Re and Im rows per k1      rows [k1][2][n2]  cols [k1][2][n2][x]
//   Z  the inverse's input, read as [2][a1][a2]  rows [2][k]       cols [2][k][x]
// Every size is a power of two and is passed as its base-2 logarithm; all
// flat indices of one buffer fit 32 bits (at most 2^30 values).
#pragma once
#include <stdint.h>

namespace ccm {

// Epilogues of the matrix-core product (k_gemm_bf16x3, gemm_mfma.hpp).
enum FsEpilogue {
  EPI_STORE = 0,     // C(m, n) at c[n ldc + m]
  EPI_TW_M,          // step 2 on step 1's output, n2 = m (rows)
  EPI_TW_Z,          // step 2, n2 = the batch entry (columns, one field per launch)
  EPI_POST_ROWS,     // forward step 3's outputs into natural order (rows)
  EPI_POST_COLS,     // the same along y (columns)
  EPI_IPOST_ROWS,    // inverse step 3's outputs into x order (rows)
  EPI_IPOST_COLS,    // the same along y (columns)
};
// The row-direction epilogues of step 3 take the MFMA operands the other way
// round (m along the accumulator rows, n along the lanes), so that the lanes
// of a store run along k1 (b1), contiguous in the output line.
__host__ __device__ constexpr bool fs_swapped(int epi) {
  return epi == EPI_POST_ROWS || epi == EPI_IPOST_ROWS;
}

struct FsArgs {
  int l1, l2;            // log2 N1, log2 N2
  int lx;                // log2 nx (columns)
  const float2* tw;      // step 2's factors, [k1][n2]
};

// Position in x of v_m.
__device__ __forceinline__ uint32_t fs_place(uint32_t m, uint32_t n) {
  return m < n / 2 ? 2 * m : 2 * (n - 1 - m) + 1;
}

// Elements (m, n) and (m, n + 1) of batch entry z of a product's result (or
// (m, n) and (m + 1, n) with the operands swapped), stored through the
// epilogue EPI. For the twiddles c points at the entry's output; for the
// others at the whole output.
template <int EPI>
__device__ __forceinline__ void fs_epilogue(float* __restrict__ c, int ldc, uint32_t z,
                                            uint32_t m, uint32_t n, float x0, float x1,
                                            const FsArgs& f) {
  const int ln = f.l1 + f.l2;
  const uint32_t nn = 1u << ln, n1m = (1u << f.l1) - 1;
  if constexpr (EPI == EPI_TW_M || EPI == EPI_TW_Z) {
    // (x0, x1) = (Re, Im) at rows n = 2 k1, 2 k1 + 1
    const uint32_t n2 = EPI == EPI_TW_M ? m : z;
    const float2 w = f.tw[((n >> 1) << f.l2) + n2];
    c[(size_t)n * ldc + m] = x0 * w.x - x1 * w.y;
    c[(size_t)(n + 1) * ldc + m] = x0 * w.y + x1 * w.x;
  } else if constexpr (EPI == EPI_POST_ROWS) {
    // y_k at k2 = m, m + 1 (k = k1 + N1 k2), n = line N1 + k1
    const uint32_t k = (n & n1m) + (m << f.l1);
    float* y = c + ((size_t)(n >> f.l1) << ln);
    y[k] = k == 0 ? x0 * 0.70710678118654752f : x0;
    y[k + (1u << f.l1)] = x1;
  } else if constexpr (EPI == EPI_POST_COLS) {
    // y_k at k2 = n, n + 1; z = field N1 + k1; m = column
    const uint32_t k = (z & n1m) + (n << f.l1);
    float* y = c + ((size_t)(z >> f.l1) << (ln + f.lx)) + m;
    y[(size_t)k << f.lx] = k == 0 ? x0 * 0.70710678118654752f : x0;
    y[(size_t)(k + (1u << f.l1)) << f.lx] = x1;
  } else if constexpr (EPI == EPI_IPOST_ROWS) {
    // v at b2 = m, m + 1; n = line N1 + b1
    float* xo = c + ((size_t)(n >> f.l1) << ln);
    const uint32_t b1 = n & n1m;
    xo[fs_place(b1 + (m << f.l1), nn)] = x0;
    xo[fs_place(b1 + ((m + 1) << f.l1), nn)] = x1;
  } else if constexpr (EPI == EPI_IPOST_COLS) {
    // v at b2 = n, n + 1; z = field N1 + b1; m = column
    float* xo = c + ((size_t)(z >> f.l1) << (ln + f.lx)) + m;
    const uint32_t b1 = z & n1m;
    xo[(size_t)fs_place(b1 + (n << f.l1), nn) << f.lx] = x0;
    xo[(size_t)fs_place(b1 + ((n + 1) << f.l1), nn) << f.lx] = x1;
  }
}

// ---- step 0 and the reordering, in step 1's operand loader ------------------------

// How step 1 reads its data operand (column mode: element (k, m) of batch entry z).
enum FsLoad {
  XL_PLAIN = 0,        // x[z sx + k ldx + m]
  XL_MAKHOUL_ROWS,     // reordered line z: v[k N2 + m] = x[z N + src(k N2 + m)]
  XL_MAKHOUL_COLS,     // reordered rows: v[(k N2 + z) nx + m] = x[src(k N2 + z) nx + m]
  XL_Z_ROWS,           // step 0 of line z: Z[re/im][k' N2 + m], k = re/im N1 + k'
  XL_Z_COLS,           // step 0 along y: Z[re/im][(k' N2 + z) nx + m]
};

// Makhoul source index of position j of the reordered line.
__device__ __forceinline__ uint32_t fs_src(uint32_t j, uint32_t n) {
  return j < n / 2 ? 2 * j : 2 * (n - 1 - j) + 1;
}

// Step 0 at natural index j of a line whose element i is at y[i * stride]:
// the real part (re) or the imaginary part.
__device__ __forceinline__ float fs_z(const float* __restrict__ y, uint32_t j, bool im,
                                      uint32_t n, uint32_t stride) {
  if (!im) return j == 0 ? y[0] * 1.41421356237309505f : y[(size_t)j * stride];
  return j == 0 ? 0.0f : y[(size_t)(n - j) * stride];
}

// Element (k, m) of batch entry z of step 1's data operand; x is the whole
// input (not offset by the batch entry).
template <int XL>
__device__ __forceinline__ float fs_load(const float* __restrict__ x, uint32_t z, uint32_t k,
                                         uint32_t m, const FsArgs& f) {
  const int ln = f.l1 + f.l2;
  const uint32_t n = 1u << ln, n1m = (1u << f.l1) - 1;
  if constexpr (XL == XL_MAKHOUL_ROWS) {
    return x[((size_t)z << ln) + fs_src((k << f.l2) + m, n)];
  } else if constexpr (XL == XL_MAKHOUL_COLS) {
    return x[((size_t)fs_src((k << f.l2) + z, n) << f.lx) + m];
  } else if constexpr (XL == XL_Z_ROWS) {
    return fs_z(x + ((size_t)z << ln), ((k & n1m) << f.l2) + m, k > n1m, n, 1);
  } else {
    return fs_z(x + m, ((k & n1m) << f.l2) + z, k > n1m, n, 1u << f.lx);
  }
}

}  // namespace ccm
