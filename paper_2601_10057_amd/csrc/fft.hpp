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

#include "lds_swizzle.hpp"

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

// LDS layout of a buffer of lines: element x lives at x ^ T(x >> B), with T a
// linear map over GF(2) from the bits above B into the low B bits (B = 5 for
// 8-byte, 4 for 16-byte elements), so that 2^B consecutive slots always cover
// all 64 banks. T is chosen per element size, line length and kernel class
// (tables in lds_swizzle.hpp) to keep the FFT stages, the Makhoul-ordered
// loads and the digit-reversed reads free of bank conflicts. Being linear,
// at(a ^ b) = at(a) ^ at(b): kernels form addresses as a per-thread base XOR
// a compile-time constant.
template <typename T, int N, int CLS> struct LdsMap {
  using Tab = SwzTab<(int)sizeof(cpx<T>), N, CLS>;
  static constexpr int B = sizeof(cpx<T>) == 8 ? 5 : 4;
  __host__ __device__ static constexpr int at(int x) {
    int r = x;
#pragma unroll
    for (int b = 0; b < Tab::NC; ++b) r ^= ((x >> (B + b)) & 1) ? Tab::col[b] : 0;
    return r;
  }
};

// Multiplies v[q] by w^q, q = 1..R-1, for w = exp(-2 pi i t / N), from one
// table lookup. FP64 lines: the powers by a running FP64 product (relative
// error about R ulp of FP64). FP32 lines: w^(2^b) by repeated FP64 squaring,
// each rounded once to FP32, and the other powers as FP32 products
// w^q = w^(q - 2^b) w^(2^b) over the lowest set bit 2^b of q (at most
// log2 R - 1 FP32 roundings per power; the transform error grows by about a
// quarter against twiddles rounded once from FP64).
template <typename T, int N, int R>
__device__ __forceinline__ void apply_twiddles(const Roots<T, N>& rt, int t, cpx<T>* v) {
  const cpx<double> w1 = rt.tw64(t);
  if constexpr (sizeof(T) == 4) {
    constexpr int LR = ilog2(R);
    cpx<T> p2[LR > 0 ? LR : 1];          // w^(2^b)
    cpx<double> w = w1;
#pragma unroll
    for (int b = 0; b < LR; ++b) {
      p2[b] = {(T)w.re, (T)w.im};
      if (b + 1 < LR) w = {w.re * w.re - w.im * w.im, 2.0 * w.re * w.im};
    }
    cpx<T> pw[R];
#pragma unroll
    for (int q = 1; q < R; ++q) {
      const int lb = q & -q;
      pw[q] = (q == lb) ? p2[ilog2(lb)] : cmul(pw[q - lb], p2[ilog2(lb)]);
      v[q] = cmul(v[q], pw[q]);
    }
  } else {
    cpx<double> w = w1;
#pragma unroll
    for (int q = 1; q < R; ++q) {
      v[q] = cmul(v[q], cpx<T>{(T)w.re, (T)w.im});
      if (q + 1 < R) w = cmul(w, w1);
    }
  }
}

// One in-place decimation-in-frequency stage over NL independent lines of
// length N stored back to back. With block length L and radix R, butterfly b
// (line b / (N/R), block j / S and offset m = j % S of j = b % (N/R), S = L/R)
// reads x[e0 + r S], e0 = line N + block L + m, forms the R-point DFT y_q and
// stores y_q exp(-2 pi i m q / L) back at x[e0 + q S]. e0 is b with log2 R
// zero bits inserted at bit log2 S, a linear map of the bits of b, so the LDS
// slots are at(e0(tid)) ^ at(e0(it NTHR)) ^ at(r S). Butterflies own disjoint
// elements; the barrier separates the stages.
template <typename T, int N, int NL, int NTHR, int R, int L, typename MAP>
__device__ __forceinline__ void dif_stage(cpx<T>* buf, const Roots<T, N>& rt, int tid) {
  constexpr int NB = N / R;
  constexpr int TOT = NB * NL;
  constexpr int S = L / R;
  constexpr int LS = ilog2(S), LR = ilog2(R);
  constexpr int ITERS = TOT >= NTHR ? TOT / NTHR : 1;
  const auto first = [](int b) { return (b & (S - 1)) | ((b >> LS) << (LS + LR)); };
  if (TOT >= NTHR || tid < TOT) {
    const int base = MAP::at(first(tid));
#pragma unroll
    for (int it = 0; it < ITERS; ++it) {
      if (ITERS > 1) __builtin_amdgcn_sched_barrier(0);   // one butterfly's registers at a time
      const int e = base ^ MAP::at(first(it * NTHR));
      const int m = (tid + it * NTHR) & (S - 1);
      cpx<T> v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = buf[e ^ MAP::at(r * S)];
      SmallDFT<T, R>::run(v);
      if (L > R) apply_twiddles<T, N, R>(rt, m * (N / L), v);
#pragma unroll
      for (int q = 0; q < R; ++q) buf[e ^ MAP::at(q * S)] = v[q];
    }
  }
  lds_sync();
}

template <typename T, int N, int NL, int NTHR, int L, bool FIRST, int RADIX, typename MAP>
struct DifRunner {
  static __device__ __forceinline__ void run(cpx<T>* buf, const Roots<T, N>& rt, int tid) {
    if constexpr (L > 1) {
      constexpr int R = FIRST ? Plan<N, RADIX>::FIRST : RADIX;
      dif_stage<T, N, NL, NTHR, R, L, MAP>(buf, rt, tid);
      DifRunner<T, N, NL, NTHR, L / R, false, RADIX, MAP>::run(buf, rt, tid);
    }
  }
};

// Forward complex FFT (exp(-2 pi i n k / N)) of NL lines in LDS, in place:
// element e of line l lives at MAP::at(l N + e); input in natural order, bin k
// found at element digit_rev<N, RADIX>(k). The caller must have synchronised
// after writing the input; the FFT ends with a barrier.
template <typename T, int N, int NL, int NTHR, int RADIX, typename MAP>
__device__ __forceinline__ void fft_lines(cpx<T>* buf, const Roots<T, N>& rt, int tid) {
  DifRunner<T, N, NL, NTHR, N, true, RADIX, MAP>::run(buf, rt, tid);
}

// Element holding DFT bin k after fft_lines: the mixed-radix digits of k
// (first radix, then the stage radix) in reverse order. For power-of-two
// radices this permutes the bits of k, so it is linear as well.
template <int N, int RADIX>
__host__ __device__ constexpr int digit_rev(int k) {
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

// Makhoul position of natural index i inside the reordered line:
// i / 2 for even i, N - 1 - (i - 1) / 2 = (N - 1) ^ (i >> 1) for odd i.
template <int N> __host__ __device__ constexpr int makhoul_slot(int i) {
  return (i & 1) ? (N - 1 - (i >> 1)) : (i >> 1);
}

// Per-thread LDS slots of the index sets a line kernel visits, thread tid of
// NTHR (a power of two) taking indices tid + q NTHR:
//   nat(q)   natural element k,                    at(k)
//   mak(q)   Makhoul slot of natural index i,      at(makhoul_slot(i))
//   bin(q)   bin k after the forward FFT,          at(digit_rev(k))
//   out(q)   natural index i after the inverse,    at(digit_rev(makhoul_slot(i)))
// and, for pair units u = tid + q NTHR < N/2 (bins u and N - u, unit 0 taking
// bins 0 and N/2), the slots of the second bin in natural and digit-reversed
// order. Each is a base XOR a constant (N - u = (N - 1) ^ (u - 1), and the
// maps are linear); lane 0 of the pair sets takes constants.
template <int N, int NTHR, int RADIX, typename MAP> struct LineSlots {
  static __host__ __device__ constexpr int g(int k) { return MAP::at(digit_rev<N, RADIX>(k)); }
  int nat0, mak0, bin0, out0, natm0, binm0;
  bool lane0;
  __device__ __forceinline__ explicit LineSlots(int tid) {
    const int t = tid & (NTHR - 1);
    lane0 = (t == 0);
    nat0 = MAP::at(t);
    mak0 = MAP::at(t >> 1) ^ ((t & 1) ? MAP::at(N - 1) : 0);
    bin0 = g(t);
    out0 = g(t >> 1) ^ ((t & 1) ? MAP::at(N - 1) : 0);
    natm0 = MAP::at(N - 1) ^ MAP::at((t - 1) & (N - 1));
    binm0 = MAP::at(N - 1) ^ g((t - 1) & (N - 1));
  }
  template <int Q> __device__ __forceinline__ int nat() const { return nat0 ^ MAP::at(Q * NTHR); }
  template <int Q> __device__ __forceinline__ int mak() const {
    return mak0 ^ MAP::at(Q * (NTHR / 2));
  }
  template <int Q> __device__ __forceinline__ int bin() const { return bin0 ^ g(Q * NTHR); }
  template <int Q> __device__ __forceinline__ int out() const { return out0 ^ g(Q * (NTHR / 2)); }
  // second bin of pair unit tid + Q NTHR
  template <int Q> __device__ __forceinline__ int natm() const {
    constexpr int c0 = Q == 0 ? MAP::at(N / 2)
                              : (MAP::at(N - 1) ^ MAP::at((Q * NTHR - 1) & (N - 1)));
    return lane0 ? c0 : (natm0 ^ MAP::at(Q * NTHR));
  }
  template <int Q> __device__ __forceinline__ int binm() const {
    constexpr int c0 = Q == 0 ? g(N / 2) : (MAP::at(N - 1) ^ g((Q * NTHR - 1) & (N - 1)));
    return lane0 ? c0 : (binm0 ^ g(Q * NTHR));
  }
};

// Bin index of the second member of pair unit u.
template <int N> __device__ __forceinline__ int pair_mirror(int u) { return u ? N - u : N / 2; }

// Orthonormal DCT-II coefficients of lines a and b (FFT of z = v_a + i v_b in
// Makhoul order) at bin k from Z_k, Z_{N-k}, w = exp(-i pi k / (2N)) and the
// scale s_k / 2.
template <typename T>
__device__ __forceinline__ void dct2_bin(cpx<T> z, cpx<T> zm, cpx<T> w, T s, T& A, T& B) {
  const T v1r = z.re + zm.re, v1i = z.im - zm.im;
  const T v2r = z.im + zm.im, v2i = zm.re - z.re;
  A = s * (w.re * v1r - w.im * v1i);
  B = s * (w.re * v2r - w.im * v2i);
}

// Both bins of a pair unit u > 0 from Z_u and Z_{N-u}: with p = w_u v1 and
// r = w_u v2, A_u = s Re p, A_{N-u} = -s Im p (and B likewise), because
// w_{N-u} = -i conj(w_u) and the mirror bin sees conj(v1), conj(v2).
template <typename T>
__device__ __forceinline__ void dct2_pair(cpx<T> z, cpx<T> zm, cpx<T> w, T s, T& A, T& B,
                                          T& Am, T& Bm) {
  const T v1r = z.re + zm.re, v1i = z.im - zm.im;
  const T v2r = z.im + zm.im, v2i = zm.re - z.re;
  A = s * (w.re * v1r - w.im * v1i);
  Am = -s * (w.re * v1i + w.im * v1r);
  B = s * (w.re * v2r - w.im * v2i);
  Bm = -s * (w.re * v2i + w.im * v2r);
}

// DCT-II post-processing of pair unit u (bins u and pair_mirror(u)) from the
// FFT output at slots pk (bin u) and pm (its mirror).
template <typename T, int N>
__device__ __forceinline__ void dct2_unit(const cpx<T>* Z, int pk, int pm, const Roots<T, N>& rt,
                                          int u, T& A, T& B, T& Am, T& Bm) {
  const cpx<T> z = Z[pk];
  const cpx<T> zm = Z[pm];
  const T s1 = (T)(0.5 * sqrt(2.0 / N));
  if (u != 0) {
    dct2_pair<T>(z, zm, rt.omega(u), s1, A, B, Am, Bm);
  } else {
    const T s0 = (T)(0.5 * sqrt(1.0 / N));
    dct2_bin<T>(z, z, cpx<T>{(T)1, (T)0}, s0, A, B);
    dct2_bin<T>(zm, zm, rt.omega(N / 2), s1, Am, Bm);
  }
}

// DCT-III pre-processing: from the orthonormal coefficients of two lines at
// bins k and N - k (A_k, A_{N-k}, B_k, B_{N-k}) build the conjugated,
// 1/N-scaled input of the forward FFT whose output y gives a[pi(n)] = Re y_n,
// b[pi(n)] = -Im y_n. For a pair unit u > 0 one set of products gives both
// Z_u and Z_{N-u}: with c = conj(w_u), v1 = c (x1 - i x1m), v2 = c (x2 - i x2m),
//   Z_u = (v1r - v2i, -(v1i + v2r)),  Z_{N-u} = (v1r + v2i, v1i - v2r).
template <typename T, int N>
__device__ __forceinline__ void dct3_pair(const Roots<T, N>& rt, int u, T Ak, T Akm, T Bk, T Bkm,
                                          cpx<T>& Z, cpx<T>& Zm) {
  const T g0 = (T)(sqrt((double)N) / N);          // 1 / (N s_0)
  const T g1 = (T)(sqrt(0.5 * N) / N);            // 1 / (N s_k), k > 0
  if (u != 0) {
    const T x1 = Ak * g1, x2 = Bk * g1, x1m = Akm * g1, x2m = Bkm * g1;
    const cpx<T> w = rt.omega(u);
    const T cr = w.re, ci = -w.im;
    const T v1r = cr * x1 + ci * x1m, v1i = ci * x1 - cr * x1m;
    const T v2r = cr * x2 + ci * x2m, v2i = ci * x2 - cr * x2m;
    Z = {v1r - v2i, -(v1i + v2r)};
    Zm = {v1r + v2i, v1i - v2r};
  } else {
    // bin 0 (no mirror partner) and bin N/2 (its own mirror)
    Z = {Ak * g0, -(Bk * g0)};
    const T x1 = Akm * g1, x2 = Bkm * g1;
    const cpx<T> w = rt.omega(N / 2);
    const T cr = w.re, ci = -w.im;
    const T v1r = (cr + ci) * x1, v1i = (ci - cr) * x1;
    const T v2r = (cr + ci) * x2, v2i = (ci - cr) * x2;
    Zm = {v1r - v2i, -(v1i + v2r)};
  }
}

}  // namespace ccm
