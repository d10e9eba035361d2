// Block-cooperative FFT and two-for-one DCT-II / DCT-III on LDS lines (gfx950).
//
// The fast direct solver of the paper (App. C) needs orthonormal 2D DCTs of
// cell-centred fields with homogeneous Neumann boundaries. A length-N DCT-II
// of a real line x is computed with Makhoul's reordering
//     v_n = x_{2n},  v_{N-1-n} = x_{2n+1},  V = DFT_N(v),
//     X_k = s_k Re(exp(-i pi k / (2N)) V_k),  s_0 = sqrt(1/N), s_k = sqrt(2/N),
// and two real lines a, b share one complex FFT of z = v_a + i v_b
// (V_a = (Z_k + conj Z_{-k})/2, V_b = (Z_k - conj Z_{-k})/(2i)). The DCT-III
// runs the same steps backwards. The complex FFT is an in-place
// decimation-in-frequency transform in LDS (radix-8 butterflies in registers,
// digit-reversed output).
#pragma once
#include <hip/hip_runtime.h>

namespace ccm {

template <typename T> struct cpx { T re, im; };

template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// exp(-2 pi i k / 16), k = 0..7, from cos/sin of multiples of pi/8.
__host__ __device__ constexpr double w16re(int k) {
  constexpr double t[8] = {1.0, 0.9238795325112867561282, 0.7071067811865475244008,
                           0.3826834323650897717285, 0.0, -0.3826834323650897717285,
                           -0.7071067811865475244008, -0.9238795325112867561282};
  return t[k];
}
__host__ __device__ constexpr double w16im(int k) {
  constexpr double t[8] = {0.0, -0.3826834323650897717285, -0.7071067811865475244008,
                           -0.9238795325112867561282, -1.0, -0.9238795325112867561282,
                           -0.7071067811865475244008, -0.3826834323650897717285};
  return t[k];
}

// In-register DFT of size R (decimation in time, recursive on R/2).
template <typename T, int R> struct SmallDFT {
  static __device__ __forceinline__ void run(cpx<T>* v) {
    constexpr int H = R / 2;
    cpx<T> e[H], o[H];
#pragma unroll
    for (int i = 0; i < H; ++i) { e[i] = v[2 * i]; o[i] = v[2 * i + 1]; }
    SmallDFT<T, H>::run(e);
    SmallDFT<T, H>::run(o);
#pragma unroll
    for (int k = 0; k < H; ++k) {
      cpx<T> t;
      constexpr int step = 16 / R;
      if (k == 0) {
        t = o[k];
      } else if (2 * k == H) {                 // multiply by -i
        t = {o[k].im, -o[k].re};
      } else {
        const T wr = (T)w16re(k * step), wi = (T)w16im(k * step);
        t = {o[k].re * wr - o[k].im * wi, o[k].re * wi + o[k].im * wr};
      }
      v[k] = {e[k].re + t.re, e[k].im + t.im};
      v[k + H] = {e[k].re - t.re, e[k].im - t.im};
    }
  }
};
template <typename T> struct SmallDFT<T, 1> {
  static __device__ __forceinline__ void run(cpx<T>*) {}
};

// Roots of unity omega(m) = exp(-2 pi i m / (4N)) from two short tables in LDS:
// omega(m) = hi[m >> S] * lo[m & (2^S - 1)], both entries from sincospi in FP64.
template <typename T, int N> struct Roots {
  static constexpr int M = 4 * N;
  static constexpr int LOGM = ilog2(M);
  static constexpr int S = (LOGM + 1) / 2;
  static constexpr int NLO = 1 << S;
  static constexpr int NHI = M >> S;
  static constexpr int SIZE = NLO + NHI;     // complex entries of LDS needed
  cpx<T>* lo;
  cpx<T>* hi;

  __device__ void init(cpx<T>* smem, int tid, int nthr) {
    lo = smem;
    hi = smem + NLO;
    for (int q = tid; q < NLO; q += nthr) {
      double s, c;
      sincospi(-2.0 * (double)q / (double)M, &s, &c);
      lo[q] = {(T)c, (T)s};
    }
    for (int q = tid; q < NHI; q += nthr) {
      double s, c;
      sincospi(-2.0 * (double)q * (double)NLO / (double)M, &s, &c);
      hi[q] = {(T)c, (T)s};
    }
  }
  __device__ __forceinline__ cpx<T> omega(int m) const {
    return cmul(hi[m >> S], lo[m & (NLO - 1)]);
  }
  // exp(-2 pi i m / N)
  __device__ __forceinline__ cpx<T> tw(int m) const { return omega(4 * m); }
};

// Radix plan: radix-8 stages, with one smaller stage first when log2 N is not
// a multiple of 3.
template <int N> struct Plan {
  static constexpr int LOGN = ilog2(N);
  static constexpr int FIRST = (LOGN % 3 == 0) ? 8 : (LOGN % 3 == 1 ? 2 : 4);
};

// One in-place decimation-in-frequency stage over NL independent lines of
// length N stored back to back. With block length L and radix R, butterfly m
// of a block reads x[m + r L/R] (r < R), forms the R-point DFT y_q and stores
// y_q exp(-2 pi i m q / L) back at x[m + q L/R]. Butterflies own disjoint
// positions, so a thread handles its butterflies one after another with only
// R values live; the barrier separates the stages.
template <typename T, int N, int NL, int NTHR, int R, int L>
__device__ __forceinline__ void dif_stage(cpx<T>* buf, const Roots<T, N>& rt, int tid) {
  constexpr int NB = N / R;
  constexpr int TOT = NB * NL;
  constexpr int S = L / R;
  for (int b = tid; b < TOT; b += NTHR) {
    const int line = b / NB, jb = b % NB;
    const int blk = jb / S, m = jb % S;
    cpx<T>* x = buf + line * N + blk * L + m;
    cpx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = x[r * S];
    SmallDFT<T, R>::run(v);
    if (L > R) {
#pragma unroll
      for (int q = 1; q < R; ++q) v[q] = cmul(v[q], rt.tw(m * q * (N / L)));
    }
#pragma unroll
    for (int q = 0; q < R; ++q) x[q * S] = v[q];
  }
  __syncthreads();
}

template <typename T, int N, int NL, int NTHR, int L, bool FIRST>
struct DifRunner {
  static __device__ __forceinline__ void run(cpx<T>* buf, const Roots<T, N>& rt, int tid) {
    if constexpr (L > 1) {
      constexpr int R = FIRST ? Plan<N>::FIRST : 8;
      dif_stage<T, N, NL, NTHR, R, L>(buf, rt, tid);
      DifRunner<T, N, NL, NTHR, L / R, false>::run(buf, rt, tid);
    }
  }
};

// Forward complex FFT (exp(-2 pi i n k / N)) of NL lines in LDS, in place:
// natural order in, bin k found at fft_pos<N>(k) out. The caller must have
// synchronised after writing the input; the FFT ends with a barrier.
template <typename T, int N, int NL, int NTHR>
__device__ __forceinline__ void fft_lines(cpx<T>* buf, const Roots<T, N>& rt, int tid) {
  DifRunner<T, N, NL, NTHR, N, true>::run(buf, rt, tid);
}

// Position of DFT bin k after fft_lines: the mixed-radix digits of k
// (first radix, then radix 8) in reverse order.
template <int N> __device__ __forceinline__ int fft_pos(int k) {
  constexpr int R1 = Plan<N>::FIRST;
  constexpr int LR1 = ilog2(R1);
  constexpr int ND = (Plan<N>::LOGN - LR1) / 3;
  int span = N / R1;
  int p = (k & (R1 - 1)) * span;
  k >>= LR1;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    span >>= 3;
    p += (k & 7) * span;
    k >>= 3;
  }
  return p;
}

// Makhoul position of natural index i inside the reordered line.
template <int N> __device__ __forceinline__ int makhoul_slot(int i) {
  return (i & 1) ? (N - 1 - (i >> 1)) : (i >> 1);
}
// Natural index stored at reordered slot n.
template <int N> __device__ __forceinline__ int makhoul_index(int n) {
  return (n < N / 2) ? 2 * n : 2 * (N - 1 - n) + 1;
}

// DCT-II post-processing of bin k after fft_lines of z = v_a + i v_b:
// returns the orthonormal coefficients A_k (line a) and B_k (line b).
template <typename T, int N>
__device__ __forceinline__ void dct2_post(const cpx<T>* Z, const Roots<T, N>& rt, int k,
                                          T& A, T& B) {
  const cpx<T> z = Z[fft_pos<N>(k)];
  const cpx<T> zm = Z[fft_pos<N>((N - k) & (N - 1))];
  const T s = (k == 0) ? (T)(0.5 * sqrt(1.0 / N)) : (T)(0.5 * sqrt(2.0 / N));
  const T v1r = z.re + zm.re, v1i = z.im - zm.im;
  const T v2r = z.im + zm.im, v2i = zm.re - z.re;
  const cpx<T> w = rt.omega(k);
  A = s * (w.re * v1r - w.im * v1i);
  B = s * (w.re * v2r - w.im * v2i);
}

// DCT-III pre-processing of bin k: from the orthonormal coefficients of two
// lines (A_k, A_{N-k}, B_k, B_{N-k}) build the conjugated, 1/N-scaled input of
// the forward FFT whose output y gives a[pi(n)] = Re y_n, b[pi(n)] = -Im y_n.
template <typename T, int N>
__device__ __forceinline__ cpx<T> dct3_pre(const Roots<T, N>& rt, int k, T Ak, T Akm, T Bk,
                                           T Bkm) {
  const T g0 = (T)(sqrt((double)N) / N);          // 1 / (N s_0)
  const T g1 = (T)(sqrt(0.5 * N) / N);            // 1 / (N s_k), k > 0
  T x1, x1m, x2, x2m;
  if (k == 0) {
    x1 = Ak * g0; x2 = Bk * g0; x1m = 0; x2m = 0;
  } else {
    x1 = Ak * g1; x2 = Bk * g1; x1m = Akm * g1; x2m = Bkm * g1;
  }
  const cpx<T> w = rt.omega(k);            // conj(w) multiplies (X - i X_{N-k})
  const T cr = w.re, ci = -w.im;
  const T v1r = cr * x1 + ci * x1m, v1i = ci * x1 - cr * x1m;
  const T v2r = cr * x2 + ci * x2m, v2i = ci * x2 - cr * x2m;
  return {v1r - v2i, -(v1i + v2r)};
}

}  // namespace ccm
