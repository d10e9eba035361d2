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

// Workgroup barrier for LDS traffic only: waits for this wave's LDS operations
// and synchronises the workgroup, while global loads and stores stay in flight
// (__syncthreads() would first wait for all of them). The kernels never pass
// data between the threads of a workgroup through global memory.
__device__ __forceinline__ void lds_sync() {
  __asm__ volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

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

// Roots of unity omega(m) = exp(-2 pi i m / (4N)) from two short FP64 tables in
// LDS: omega(m) = hi[m >> S] * lo[m & (2^S - 1)], entries from sincospi.
template <typename T, int N> struct Roots {
  static constexpr int M = 4 * N;
  static constexpr int LOGM = ilog2(M);
  static constexpr int S = (LOGM + 1) / 2;
  static constexpr int NLO = 1 << S;
  static constexpr int NHI = M >> S;
  static constexpr int SIZE = NLO + NHI;     // FP64 complex entries of LDS needed
  cpx<double>* lo;
  cpx<double>* hi;

  __device__ void init(cpx<double>* smem, int tid, int nthr) {
    lo = smem;
    hi = smem + NLO;
    for (int q = tid; q < NLO; q += nthr) {
      double s, c;
      sincospi(-2.0 * (double)q / (double)M, &s, &c);
      lo[q] = {c, s};
    }
    for (int q = tid; q < NHI; q += nthr) {
      double s, c;
      sincospi(-2.0 * (double)q * (double)NLO / (double)M, &s, &c);
      hi[q] = {c, s};
    }
  }
  __device__ __forceinline__ cpx<double> omega64(int m) const {
    return cmul(hi[m >> S], lo[m & (NLO - 1)]);
  }
  __device__ __forceinline__ cpx<T> omega(int m) const {
    const cpx<double> w = omega64(m);
    return {(T)w.re, (T)w.im};
  }
  // exp(-2 pi i m / N) in FP64
  __device__ __forceinline__ cpx<double> tw64(int m) const { return omega64(4 * m); }
};

// Radix of the FFT stages: 16 for FP32 lines, 8 for FP64 lines (register
// budget of one butterfly).
template <typename T> constexpr int fft_radix() { return sizeof(T) == 4 ? 16 : 8; }

// Stage plan: radix-RADIX stages with one smaller stage first when log2 N is
// not a multiple of log2 RADIX.
template <int N, int RADIX> struct Plan {
  static constexpr int LOGN = ilog2(N);
  static constexpr int LR = ilog2(RADIX);
  static constexpr int REM = LOGN % LR;
  static constexpr int FIRST = REM == 0 ? RADIX : (1 << REM);
};

// LDS position of element e of a line: an XOR swizzle inside aligned groups of
// 32 elements that keeps every FFT stage, including the short-stride last
// ones, free of bank conflicts for 8- and 16-byte elements.
__device__ __forceinline__ int lds_pos(int e) { return e ^ ((e >> 5) & 31); }

// Multiplies v[q] by w^q, q = 1..R-1, for w = exp(-2 pi i t / N): one table
// lookup, then the powers by a running FP64 product (relative error about
// R ulp of FP64), each rounded to T.
template <typename T, int N, int R>
__device__ __forceinline__ void apply_twiddles(const Roots<T, N>& rt, int t, cpx<T>* v) {
  const cpx<double> w1 = rt.tw64(t);
  cpx<double> w = w1;
#pragma unroll
  for (int q = 1; q < R; ++q) {
    v[q] = cmul(v[q], cpx<T>{(T)w.re, (T)w.im});
    if (q + 1 < R) w = cmul(w, w1);
  }
}

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
    cpx<T>* x = buf + line * N;
    const int e0 = blk * L + m;
    cpx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = x[lds_pos(e0 + r * S)];
    SmallDFT<T, R>::run(v);
    if (L > R) apply_twiddles<T, N, R>(rt, m * (N / L), v);
#pragma unroll
    for (int q = 0; q < R; ++q) x[lds_pos(e0 + q * S)] = v[q];
  }
  lds_sync();
}

template <typename T, int N, int NL, int NTHR, int L, bool FIRST, int RADIX>
struct DifRunner {
  static __device__ __forceinline__ void run(cpx<T>* buf, const Roots<T, N>& rt, int tid) {
    if constexpr (L > 1) {
      constexpr int R = FIRST ? Plan<N, RADIX>::FIRST : RADIX;
      dif_stage<T, N, NL, NTHR, R, L>(buf, rt, tid);
      DifRunner<T, N, NL, NTHR, L / R, false, RADIX>::run(buf, rt, tid);
    }
  }
};

// Forward complex FFT (exp(-2 pi i n k / N)) of NL lines in LDS, in place:
// element e of a line lives at lds_pos(e); input in natural order, bin k found
// at bin_pos<T, N>(k). The caller must have synchronised after writing the
// input; the FFT ends with a barrier.
template <typename T, int N, int NL, int NTHR, int RADIX = fft_radix<T>()>
__device__ __forceinline__ void fft_lines(cpx<T>* buf, const Roots<T, N>& rt, int tid) {
  DifRunner<T, N, NL, NTHR, N, true, RADIX>::run(buf, rt, tid);
}

// Position of DFT bin k after fft_lines (before the swizzle): the mixed-radix
// digits of k (first radix, then the stage radix) in reverse order.
template <typename T, int N, int RADIX = fft_radix<T>()>
__device__ __forceinline__ int fft_pos(int k) {
  using P = Plan<N, RADIX>;
  constexpr int R1 = P::FIRST;
  constexpr int LR1 = ilog2(R1);
  constexpr int ND = (P::LOGN - LR1) / P::LR;
  int span = N / R1;
  int p = (k & (R1 - 1)) * span;
  k >>= LR1;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    span >>= P::LR;
    p += (k & (RADIX - 1)) * span;
    k >>= P::LR;
  }
  return p;
}

// LDS position of bin k after fft_lines.
template <typename T, int N, int RADIX = fft_radix<T>()>
__device__ __forceinline__ int bin_pos(int k) {
  return lds_pos(fft_pos<T, N, RADIX>(k));
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
// What the DCT-II post-processing of bin k needs besides the line itself:
// the LDS positions of bins k and N - k, the twiddle and the scale. Lines of
// the same length share it.
template <typename T> struct PostTerm {
  int pk, pm;
  cpx<T> w;
  T s;
};

template <typename T, int N, int RADIX = fft_radix<T>()>
__device__ __forceinline__ PostTerm<T> dct2_term(const Roots<T, N>& rt, int k) {
  PostTerm<T> t;
  t.pk = bin_pos<T, N, RADIX>(k);
  t.pm = bin_pos<T, N, RADIX>((N - k) & (N - 1));
  t.w = rt.omega(k);
  t.s = (k == 0) ? (T)(0.5 * sqrt(1.0 / N)) : (T)(0.5 * sqrt(2.0 / N));
  return t;
}

template <typename T>
__device__ __forceinline__ void dct2_post(const cpx<T>* Z, const PostTerm<T>& t, T& A, T& B) {
  const cpx<T> z = Z[t.pk];
  const cpx<T> zm = Z[t.pm];
  const T v1r = z.re + zm.re, v1i = z.im - zm.im;
  const T v2r = z.im + zm.im, v2i = zm.re - z.re;
  A = t.s * (t.w.re * v1r - t.w.im * v1i);
  B = t.s * (t.w.re * v2r - t.w.im * v2i);
}

template <typename T, int N, int RADIX = fft_radix<T>()>
__device__ __forceinline__ void dct2_post(const cpx<T>* Z, const Roots<T, N>& rt, int k,
                                          T& A, T& B) {
  dct2_post<T>(Z, dct2_term<T, N, RADIX>(rt, k), A, B);
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
