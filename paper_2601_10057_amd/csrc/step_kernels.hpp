// Kernels of one CC-MSAV-BDF2 step (Sec. 3.2, solved as in App. B and App. C).
//
// Pipeline of one step (fields are row-major [ny][nx], x fastest):
//   P1a k_stencil    : the explicit stencil terms of eqs. (AC_BDF2)-(Z_BDF2) at
//       phi* = x0 phi^n + x1 phi^{n-1}: the basis numerators S~, H, Q~, K~, P~
//       (Sec. 2.2 with the discrete forms of Sec. 3.4.1), L~ = div(M_psi(A phi*)
//       grad P~), f_lin and g_lin (or their increment-form residuals), plus the
//       SAV partial sums; each wave walks down a band of rows with a register
//       window.
//   P1b k_row_dct8   : orthonormal DCT-II along x of the 8 fields for a band of
//       rows (the band's rows of a column pair leave as one piece per FP64
//       field or FP32 field pair).
//   P2  k_col_gram   : per strip of two columns, DCT-II along y and the
//       Parseval inner products (F_i, chi^{-1} F_j), (P, zeta^{-1} g), (P, zeta^{-1} L).
//   S   k_solve      : reduces the partials, assembles and solves the 5x5
//       system of App. B Step 4, updates the SAVs, and emits the spectral
//       combination coefficients (all on the device).
//   P3  k_col_solve  : per strip, combines the x-transformed fields into the
//       right-hand sides of chi phi^{n+1} and zeta psi^{n+1}, DCT-II along y,
//       divides by sigma / tau, DCT-III along y.
//   P4  k_row_idct   : per band of rows (or per row), DCT-III along x of both
//       results -> phi^{n+1}, psi^{n+1} (added to phi^n, psi^n in the
//       increment form).
// The intermediate fields use a strip-major layout: element (k, j) of a field
// lives at ((k / 2) * ny + j) * 2 + (k % 2), so that a column pair is one
// contiguous complex line. FP32 fields go two to a region, side by side in
// each row (mid_pair, step_common.hpp).
#pragma once
#include <type_traits>
#include <utility>

#include "fft.hpp"
#include "step_common.hpp"

namespace ccm {

// Calls f(std::integral_constant<int, i>{}) for i = 0 .. N-1.
template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F> __device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// The value x, which the compiler may no longer assume equal to any other
// value: expressions formed from it are computed where they are used instead
// of being shared with earlier ones and held (or spilled) in between.
__device__ __forceinline__ int opaque_vgpr(int x) {
  __asm__ volatile("" : "+v"(x));
  return x;
}

constexpr int clamp_threads(int t) { return t < 64 ? 64 : (t > 1024 ? 1024 : t); }
// Threads of a line kernel: four elements per thread.
constexpr int line_threads(int n) { return clamp_threads(n / 4); }
// Threads of a one-line kernel with one butterfly of the FFT stages per
// thread: no thread idles in the transforms and a CU holds several
// workgroups, at the price of more work per thread outside them.
template <typename TM> constexpr int one_line_threads(int n) {
  return clamp_threads(n / (sizeof(TM) == 4 ? 16 : 8));
}
template <typename TM> constexpr int line_threads_v(int n, int v) {
  return v == 0 ? line_threads(n) : one_line_threads<TM>(n);
}
// The Gram kernel keeps four spectra per thread: eight bins per thread give
// each wave up to 256 registers at one workgroup per CU. FP32 lines of 8192
// points and more take sixteen bins per thread (workgroups of 8 waves, up to
// 256 registers each) and keep their spectra in global memory.
template <typename TM> constexpr int gram_threads(int n) {
  return clamp_threads(n / (sizeof(TM) == 4 && n >= 8192 ? 16 : 8));
}
// Complex lines of length n that fit in LDS next to the twiddle tables.
template <typename TM> constexpr int lds_line_budget(int n) {
  return (136 * 1024) / (n * (int)sizeof(cpx<TM>));
}
// Rows per workgroup of the row pass. The strip-major intermediates put the
// rows of one column pair next to each other, so a workgroup holding R rows
// writes each column pair of a field as one piece of 2 R values (4 R for an
// FP32 field pair); HBM takes writes in 32-byte sectors, so R is chosen to
// fill one with a field's values (4 FP32 or 2 FP64 rows) as far as the LDS
// lines allow.
template <typename TM> constexpr int p1_rows(int n) {
  const int want = 32 / (2 * (int)sizeof(TM));
  const int fit = lds_line_budget<TM>(n);
  return fit >= want ? want : (fit >= 2 ? 2 : 1);
}
// Rows per workgroup of row inverse variant v (0: half the row pass's band,
// read as one piece per strip, with two workgroups per CU at N = 4096).
template <typename TM> constexpr int row_idct_rows(int n, int v) {
  return v == 0 ? (p1_rows<TM>(n) / 2 > 0 ? p1_rows<TM>(n) / 2 : 1) : 1;
}
// Threads of row inverse variant v: variant 0 has one FFT butterfly per
// thread over its band's lines, variant 1 over its one line.
template <typename TM> constexpr int row_idct_threads(int n, int v) {
  const int bf = row_idct_rows<TM>(n, v) * n / fft_radix<TM>();
  return v == 0 ? (bf < line_threads(n) ? clamp_threads(bf) : line_threads(n))
                : one_line_threads<TM>(n);
}
// Field pairs transformed together per round of the row pass (4 / pairs rounds).
template <typename TM> constexpr int p1_pairs(int n) {
  const int per = lds_line_budget<TM>(n) / p1_rows<TM>(n);
  return per >= 4 ? 4 : (per >= 2 ? 2 : 1);
}
// Launch variants the autotuner chooses between. Row DCT variant v halves the
// band of rows and the LDS lines v times (shorter write pieces, more
// workgroups per CU); line-kernel variant 0 has four elements per thread,
// variant 1 one FFT butterfly per thread.
template <typename TM> constexpr int p1_rows_v(int n, int v) {
  return (p1_rows<TM>(n) >> v) > 0 ? (p1_rows<TM>(n) >> v) : 1;
}
template <typename TM> constexpr int p1_pairs_v(int n, int v) {
  const int lines0 = p1_rows<TM>(n) * p1_pairs<TM>(n);
  const int lines = (lines0 >> v) > p1_rows_v<TM>(n, v) ? (lines0 >> v) : p1_rows_v<TM>(n, v);
  const int per = lines / p1_rows_v<TM>(n, v);
  return per >= 4 ? 4 : (per >= 2 ? 2 : 1);
}

// Consecutive workgroups are dispatched round-robin over the 8 XCDs; give each
// XCD a contiguous range of lines so that neighbouring rows share an L2.
__device__ __forceinline__ int xcd_remap(int b, int g) {
  if ((g & 7) != 0) return b;
  return (b & 7) * (g >> 3) + (b >> 3);
}

// Element (k, j) of a strip-major field with strip stride ss.
__device__ __forceinline__ size_t mid_index(int k, int j, size_t ss) {
  return (size_t)(k >> 1) * ss + 2 * (size_t)j + (k & 1);
}

// Element (k, j) of slot f of the strip-major intermediates of an nx x ny
// grid: one field per region (FP64), or the pair layout (FP32, mid_pair).
template <typename TM>
__device__ __forceinline__ size_t mid_offset(int f, int k, int j, int nx, int ny) {
  if constexpr (sizeof(TM) == 4)
    return mid_pair(f) * pair_field(nx, ny) + (size_t)(k >> 1) * pair_strip_stride(ny) +
           4 * (size_t)j + 2 * mid_half(f) + (k & 1);
  else
    return f * strip_field(nx, ny, sizeof(TM)) + mid_index(k, j, strip_stride(ny, sizeof(TM)));
}

// Sum NV doubles over the block in a fixed order; the totals land in red[0..NV).
template <int NV, int NTHR>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* red, int tid) {
  constexpr int NW = (NTHR + 63) / 64;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] += __shfl_xor(v[q], off, 64);
  }
  const int lane = tid & 63, w = tid >> 6;
  lds_sync();
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) red[NV + w * NV + q] = v[q];
  }
  lds_sync();
  if (tid < NV) {
    double s = 0.0;
    for (int i = 0; i < NW; ++i) s += red[NV + i * NV + tid];
    red[tid] = s;
  }
  lds_sync();
}

// The FP32-transform (mixed) path solves for the increments phi^{n+1} - phi^n and
// psi^{n+1} - psi^n: right-hand sides are residuals against the current state,
// formed in FP64, so FP32 rounding scales with the step's change rather than
// with the fields, and the mean of the psi increment is carried in FP64.
template <typename TM> constexpr bool increment_form() { return sizeof(TM) == 4; }

// Sum of buf[0..N) (N a power of two) by pairwise halving: the order of the
// additions does not depend on the number of threads, so every launch variant
// gives the same bits. Overwrites buf; starts and ends with a barrier.
template <int N> __device__ __forceinline__ double tree_sum(double* buf, int tid, int nthr) {
#pragma unroll 1
  for (int half = N / 2; half >= 1; half >>= 1) {
    lds_sync();
    for (int i = tid; i < half; i += nthr) buf[i] += buf[i + half];
  }
  lds_sync();
  return buf[0];
}

// tree_sum of ROWS rows at once, row r at buf + r RS: the same pairs per row.
template <int N, int ROWS, int RS>
__device__ __forceinline__ void tree_sum_rows(double* buf, int tid, int nthr,
                                              double (&res)[ROWS]) {
#pragma unroll 1
  for (int half = N / 2; half >= 1; half >>= 1) {
    lds_sync();
    for (int i = tid; i < ROWS * half; i += nthr) {
      const int r = i / half, k = i - r * half;
      buf[r * RS + k] += buf[r * RS + k + half];
    }
  }
  lds_sync();
#pragma unroll
  for (int r = 0; r < ROWS; ++r) res[r] = buf[r * RS];
}

// 1 / x for positive, normal x: the hardware reciprocal estimate refined by
// two Newton steps r <- r + r (1 - x r), each squaring the relative error, to
// within about 1 ulp of FP64 (cheaper than the correctly rounded division).
__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}

__device__ __forceinline__ double mobility(double phi, double M0) {
  const double t = phi * phi - 1.0;
  return 1.0 - M0 * t * t;
}

// ---------------------------------------------------------------------------
// P1: fused stencil terms + row DCT-II of the eight right-hand-side fields.
// ---------------------------------------------------------------------------
// Field pairs of the row pass (two real fields per complex FFT line).
// With FP32 intermediates they are the pairs of the layout (mid_pair), first
// half in A; FP64 keeps its own pairing (which fixes its rounding).
template <typename TM> struct RowPairs;
template <> struct RowPairs<float> {
  static constexpr int A[4] = {M_S, M_Q, M_F, M_G};
  static constexpr int B[4] = {M_H, M_K, M_P, M_L};
};
template <> struct RowPairs<double> {
  static constexpr int A[4] = {M_F, M_S, M_Q, M_L};
  static constexpr int B[4] = {M_G, M_H, M_K, M_P};
};
static_assert(mid_pair(RowPairs<float>::A[0]) == mid_pair(RowPairs<float>::B[0]) &&
                  mid_half(RowPairs<float>::B[0]) == 1 &&
                  mid_pair(RowPairs<float>::A[1]) == mid_pair(RowPairs<float>::B[1]) &&
                  mid_half(RowPairs<float>::B[1]) == 1 &&
                  mid_pair(RowPairs<float>::A[2]) == mid_pair(RowPairs<float>::B[2]) &&
                  mid_half(RowPairs<float>::B[2]) == 1 &&
                  mid_pair(RowPairs<float>::A[3]) == mid_pair(RowPairs<float>::B[3]) &&
                  mid_half(RowPairs<float>::B[3]) == 1,
              "the FP32 row pass's FFT pairs are the layout pairs");

__device__ __forceinline__ double ptilde(const StepConst& c, double psi, double p) {
  return 0.5 * (c.gamma_in * (1.0 + p) * (psi - c.psi_in) +
                c.gamma_out * (1.0 - p) * (psi - c.psi_out));
}

// Value of lane i - 1 (lane_from_below) or lane i + 1 (lane_from_above) of the
// wave, by DPP whole-wave shifts of both halves of the double; the end lanes
// get their own value back.
__device__ __forceinline__ double lane_from_below(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, 0x138, 0xf, 0xf, false),
                          __builtin_amdgcn_update_dpp(lo, lo, 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ double lane_from_above(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, 0x130, 0xf, 0xf, false),
                          __builtin_amdgcn_update_dpp(lo, lo, 0x130, 0xf, 0xf, false));
}

// P1a: the stencil terms of a band of rows. Each wave owns SW_OUT consecutive
// output columns plus two halo columns on either side (64 lanes); walking down
// the band, a lane keeps the rows above and below the current one in
// registers and takes the values at the left and right neighbours from the
// adjacent lanes, so every pointwise quantity (phi*, psi*, P~ and its sine) is
// formed once per cell. Neighbours outside the grid are the ghost copies of
// App. D (index clamping), or with periodic boundaries the cells on the other
// side of the grid (index wrapping). The eight fields are the right-hand sides of
// eqs. (AC_BDF2)-(Z_BDF2) at phi* = x0 phi^n + x1 phi^{n-1} (slot order of Mid)
// and leave row-major ([field][ny][nx], x fastest).
constexpr int STENCIL_THREADS = 256;
constexpr int SW_WAVES = STENCIL_THREADS / 64;
constexpr int SW_OUT = 60;                    // output columns per wave
constexpr int SW_COLS = SW_WAVES * SW_OUT;    // output columns per workgroup
constexpr int SW_BAND = 32;                   // rows per workgroup (ny if smaller)

// LDS of one invocation of a kernel body, its arrays gathered in one struct:
// the kernels declare one as __shared__, and the persistent step kernel
// places several side by side and reuses the space from phase to phase.
struct StencilLds {
  double red[P1_NSUM * (STENCIL_THREADS / 64 + 1)];
};
// A transform line (or band of lines) and the twiddle roots of length N.
template <typename TM, int LINE, int N> struct LinesLds {
  cpx<TM> line[LINE];
  cpx<double> rtab[Roots<TM, N>::SIZE];
};

// Launch shape of P1a for an nx x ny grid: rows per workgroup and the number
// of workgroups (one row of partial sums each). A grid of 1024 rows or more
// that would give fewer than 2048 workgroups (eight per CU) takes bands of 16
// rows instead of 32: at N = 2048 the 576 workgroups of 32-row bands left
// most CUs with two (stencil 112 us; 16-row bands 98 us, 8-row bands 97 us).
// Smaller grids keep 32 rows: they share their launches with the other
// members of an ensemble, which fill the device.
struct StencilShape {
  int iters, blocks;
};
constexpr int SW_BAND_MIN = 16;
constexpr int SW_FILL_BLOCKS = 2048;
inline StencilShape stencil_shape(int nx, int ny) {
  const int nseg = (nx + SW_COLS - 1) / SW_COLS;
  int iters = ny < SW_BAND ? ny : SW_BAND;
  if (ny >= 1024 && nseg * (ny / iters) < SW_FILL_BLOCKS && iters == SW_BAND) iters = SW_BAND_MIN;
  return {iters, nseg * (ny / iters)};
}

template <typename TM>
__device__ __forceinline__ void stencil_body(const RowArgs& a, gptr<TM> __restrict__ rm,
                                             gptr<double> __restrict__ part, int nx, int ny,
                                             int iters, const StepConst& c, int blk,
                                             gptr<double> mob_e, gptr<double> mob_n,
                                             StencilLds& L, int tid) {
  constexpr bool INC = increment_form<TM>();
  double* red = L.red;
  const int lane = tid & 63, wave = tid >> 6;
  const int nseg = (nx + SW_COLS - 1) / SW_COLS;
  const int seg = blk % nseg, band = blk / nseg;
  const int ci = seg * SW_COLS + wave * SW_OUT - 2 + lane;   // this lane's column
  const bool per = c.periodic != 0;
  // the column this lane loads: its ghost source (clamped, or wrapped)
  const int cl = per ? ((ci % nx) + nx) % nx : min(max(ci, 0), nx - 1);
  const bool out_lane = lane >= 2 && lane < 2 + SW_OUT && ci < nx;
  // Neumann ghosts at the west and east walls are the cell itself; periodic
  // neighbours are the adjacent lanes, which hold the wrapped columns
  const bool at_w = !per && ci == 0, at_e = !per && ci == nx - 1;
  const int j0 = band * iters;
  const size_t FS = (size_t)nx * ny;
  const double k32 = 0.75 * 1.4142135623730950488;   // 3 sqrt(2) / 4
  const double half_pi = 1.5707963267948966192;
  const double ieps = 1.0 / c.eps;
  // neighbour values along x (adjacent lanes, by DPP wave shifts); at the
  // boundary the ghost is the cell itself
  auto west = [&](double v) {
    const double u = lane_from_below(v);
    return at_w ? v : u;
  };
  auto east = [&](double v) {
    const double u = lane_from_above(v);
    return at_e ? v : u;
  };
  auto at = [&](int r) {
    const int rr = per ? ((r % ny) + ny) % ny : min(max(r, 0), ny - 1);
    return (size_t)rr * nx + cl;
  };

  // Pointwise quantities of one row at this column.
  struct Row {
    double phn, phm, psn, psm;    // state
    double p, q;                  // phi*, psi*
    double sp, cp, P;             // sin, cos (pi phi* / 2), P~
    double dq;                    // psi^n - psi^{n-1} (increment form)
    double dl, fl;                // lagged delta psi and phi* of the previous step
  };
  // State values of one row at this column, loaded ahead of their use.
  struct Raw {
    double phn, phm, psn, psm, psmm, phmm;
  };
  auto load_raw = [&](int r) {
    Raw w;
    const size_t o = at(r);
    w.phn = a.phn[o];
    w.phm = a.phm[o];
    w.psn = a.psn[o];
    w.psm = a.psm[o];
    if (c.lag_d) {
      w.psmm = a.psmm[o];
      w.phmm = a.phmm[o];
    } else {
      w.psmm = 0.0;
      w.phmm = 0.0;
    }
    return w;
  };
  auto make_row = [&](const Raw& v) {
    Row w;
    w.phn = v.phn;
    w.phm = v.phm;
    w.psn = v.psn;
    w.psm = v.psm;
    w.p = c.x0 * w.phn + c.x1 * w.phm;
    w.q = c.x0 * w.psn + c.x1 * w.psm;
    sincospi(0.5 * w.p, &w.sp, &w.cp);
    w.P = ptilde(c, w.q, w.sp);
    w.dq = w.psn - w.psm;
    if (c.lag_d) {
      w.dl = w.psn - 2.0 * w.psm + v.psmm;
      w.fl = 2.0 * w.phm - v.phmm;
    } else {
      w.dl = 0.0;
      w.fl = 0.0;
    }
    return w;
  };
  // Delta_h phi^n of the row whose phi^n is u, with the rows above (un) and below (us).
  auto lap_n = [&](double u, double un, double us) {
    return (east(u) + west(u) + un + us - 4.0 * u) * c.inv_h2;
  };

  double sums[P1_NSUM];
#pragma unroll
  for (int q = 0; q < P1_NSUM; ++q) sums[q] = 0.0;

  // Window: rows j-1, j, j+1 (pointwise), the raw state of row j+2, and
  // Delta_h phi^n of rows j-1, j. The loop takes four rows per trip with
  // rotating raw buffers, so that a row's loads are issued two rows before
  // their use.
  Row rs = make_row(load_raw(j0 - 1)), rc = make_row(load_raw(j0)), rn = make_row(load_raw(j0 + 1));
  double Ls = 0.0, Lc = 0.0;
  if constexpr (INC) {
    const double u2 = a.phn[at(j0 - 2)];
    Lc = lap_n(rc.phn, rn.phn, rs.phn);
    Ls = (j0 == 0) ? Lc : lap_n(rs.phn, rc.phn, u2);
  }
  // Mobility on the face below the current row: the previous row's north
  // face (the same operands in the same order, so the same value).
  double m_south = mobility(0.5 * (rs.p + rc.p), c.M0);
  auto row_step = [&](int j, const Raw& r2) {
    double Ln = 0.0;
    if constexpr (INC) Ln = (j + 1 >= ny) ? Lc : lap_n(rn.phn, r2.phn, rc.phn);
    // neighbours along x of the current row
    const double pe = east(rc.p), pw = west(rc.p);
    const double qe = east(rc.q), qw = west(rc.q);
    const double Pe = east(rc.P), Pw = west(rc.P);
    const double de = east(rc.dl), fe = east(rc.fl);
    double Le = 0.0, Lw = 0.0, dqe = 0.0, dqw = 0.0;
    if constexpr (INC) {
      Le = east(Lc);
      Lw = west(Lc);
      dqe = east(rc.dq);
      dqw = west(rc.dq);
    }
    const double pc = rc.p, pn = rn.p, ps = rs.p;
    const double gxe = (pe - pc) * c.inv_h, gxw = (pc - pw) * c.inv_h;
    const double gyn = (pn - pc) * c.inv_h, gys = (pc - ps) * c.inv_h;
    const double lap_p = (gxe - gxw + gyn - gys) * c.inv_h;
    const double pc2 = pc * pc;
    const double cubic = pc2 * pc - pc;
    const double eph = c.e0 * rc.phn + c.e1 * rc.phm;
    const double eps_ = c.e0 * rc.psn + c.e1 * rc.psm;
    double out[M_NFIELD];
    if constexpr (INC) {
      // Increment form: the residuals f_lin - chi phi^n and g_lin - zeta psi^n,
      // written so that nothing of size phi / dt or psi / dt is ever formed:
      //   a0 phi^n + a1 phi^{n-1} - alpha phi^n = -a1 (phi^n - phi^{n-1}),
      //   psi* - psi^n = (x0 - 1)(psi^n - psi^{n-1}), which carries lambda Delta;
      // Delta_h^2 phi^n is Delta_h applied to Delta_h phi^n, both with ghosts.
      const double bih = (Le + Lw + Ln + Ls - 4.0 * Lc) * c.inv_h2;
      out[M_F] = -c.a1 * (rc.phn - rc.phm) - c.C1b * rc.phn - c.M_phi * c.theta_t * lap_p +
                 c.C2 * Lc - c.C3 * bih;
      const double lap_dq = (dqe + dqw + rn.dq + rs.dq - 4.0 * rc.dq) * c.inv_h2;
      out[M_G] = -c.a1 * rc.dq - c.lam * (c.x0 - 1.0) * lap_dq;
    } else {
      out[M_F] = c.a0 * rc.phn + c.a1 * rc.phm - c.M_phi * c.theta_t * lap_p;
      double stab;
      if (c.classical) {
        // classical scheme (App. B remarks): lambda div(M_psi(phi*) grad psi*)
        const double me = mobility(0.5 * (rc.p + pe), c.M0), mw = mobility(0.5 * (pw + rc.p), c.M0);
        const double mn = mobility(0.5 * (rc.p + rn.p), c.M0);
        const double ms = mobility(0.5 * (rs.p + rc.p), c.M0);
        stab = (me * (qe - rc.q) - mw * (rc.q - qw) + mn * (rn.q - rc.q) - ms * (rc.q - rs.q)) *
               c.inv_h2;
      } else {
        stab = (qe + qw + rn.q + rs.q - 4.0 * rc.q) * c.inv_h2;
      }
      out[M_G] = c.a0 * rc.psn + c.a1 * rc.psm - c.lam * stab;
    }
    const double St = pc * (pc2 - 1.0 - c.beta) * 0.5 * ieps;
    const double Hf = k32 * (cubic * ieps - c.eps * lap_p);
    out[M_S] = St;
    out[M_H] = Hf;
    const double din = rc.q - c.psi_in, dout = rc.q - c.psi_out;
    const double fin = 0.5 * c.gamma_in * din * din + c.beta_in;
    const double fout = 0.5 * c.gamma_out * dout * dout + c.beta_out;
    const double grad2 = 0.5 * (gxe * gxe + gxw * gxw + gyn * gyn + gys * gys);
    const double div_a = 0.5 * ((pc2 + pe * pe) * gxe - (pw * pw + pc2) * gxw +
                                (pc2 + pn * pn) * gyn - (ps * ps + pc2) * gys) * c.inv_h;
    const double Qt = 6.0 * (pc * grad2 - div_a) + cubic * (3.0 * pc2 - 1.0) * ieps * ieps;
    const double Kt = 0.5 * half_pi * rc.cp * (fin - fout);
    out[M_Q] = Qt;
    out[M_K] = Kt;
    const double Pc = rc.P;
    // each face's mobility once: the west face is the west lane's east face
    // (at the west wall the ghost lane's face, mobility(phi*_0), as the
    // ghost rule gives), the south face the previous row's north face
    const double Me = mobility(0.5 * (pc + pe), c.M0), Mn = mobility(0.5 * (pc + pn), c.M0);
    const double Mw = lane_from_below(Me), Ms = m_south;
    out[M_L] = (Me * (Pe - Pc) - Mw * (Pc - Pw) + Mn * (rn.P - Pc) - Ms * (Pc - rs.P)) * c.inv_h2;
    out[M_P] = Pc;
    if (out_lane) {
      const size_t o = (size_t)j * nx + ci;
#pragma unroll
      for (int f = 0; f < M_NFIELD; ++f) rm[f * FS + o] = (TM)out[f];
      const double vq = pc2 - 1.0 - c.beta;
      sums[P1_RS] += vq * vq * 0.25 * ieps;
      sums[P1_ES] += St * eph;
      sums[P1_EH] += Hf * eph;
      sums[P1_RW] += 6.0 * pc2 * grad2 + cubic * cubic * ieps * ieps;
      sums[P1_RZ] += (1.0 + rc.sp) * fin + (1.0 - rc.sp) * fout;
      sums[P1_EQ] += Qt * eph;
      sums[P1_EK] += Kt * eph;
      sums[P1_EP] += Pc * eps_;
      if constexpr (INC) {
        sums[P1_XS] += St * rc.phn;
        sums[P1_XH] += Hf * rc.phn;
        sums[P1_XQ] += Qt * rc.phn;
        sums[P1_XK] += Kt * rc.phn;
        sums[P1_XP] += Pc * rc.psn;
      }
      // the east and north faces of the cell (with periodic boundaries the
      // faces across the wrap belong to the last column and row)
      const bool face_e = per || ci < nx - 1, face_n = per || j < ny - 1;
      if (face_e && !(Me > 0.0)) sums[P1_MOBNEG] += 1.0;
      if (face_n && !(Mn > 0.0)) sums[P1_MOBNEG] += 1.0;
      if (c.classical) {
        sums[P1_MBAR] += mobility(pc, c.M0);
        mob_e[o] = face_e ? Me : 0.0;
        mob_n[o] = face_n ? Mn : 0.0;
      }
      if (c.lag_d) {
        // ||d^n||^2 of the previous step over the east and north faces
        if (face_e) {
          const double g = de - rc.dl;
          sums[P1_DLAG] += g * g * c.inv_h2 * rcp64(mobility(0.5 * (rc.fl + fe), c.M0));
        }
        if (face_n) {
          const double g = rn.dl - rc.dl;
          sums[P1_DLAG] += g * g * c.inv_h2 * rcp64(mobility(0.5 * (rc.fl + rn.fl), c.M0));
        }
      }
    }
    // advance the window
    m_south = Mn;
    rs = rc;
    rc = rn;
    if (j + 1 < j0 + iters) rn = make_row(r2);
    Ls = Lc;
    Lc = Ln;
  };
  Raw r0 = load_raw(j0 + 2), r1 = load_raw(j0 + 3);
#pragma unroll 1
  for (int j = j0; j < j0 + iters; j += 4) {
    const Raw r2 = load_raw(j + 4);
    row_step(j, r0);
    const Raw r3 = load_raw(j + 5);
    row_step(j + 1, r1);
    if (j + 4 < j0 + iters) r0 = load_raw(j + 6);
    row_step(j + 2, r2);
    if (j + 4 < j0 + iters) r1 = load_raw(j + 7);
    row_step(j + 3, r3);
  }
  block_sum<P1_NSUM, STENCIL_THREADS>(sums, red, tid);
  if (tid < P1_NSUM) part[(size_t)blk * P1_NSUM + tid] = red[tid];
}

// Column-pair piece of one field over the rows of a workgroup, stored with one
// wide write.
template <typename TM, int ROWS> struct alignas(2 * ROWS * sizeof(TM)) RowPiece {
  TM v[2 * ROWS];
};

// Complex values in global memory, moved field by field (the address-space
// qualified element has no implicit copy).
template <typename T> __device__ __forceinline__ cpx<T> gload(gptr<const cpx<T>> p) {
  return {p->re, p->im};
}
template <typename T> __device__ __forceinline__ void gstore(gptr<cpx<T>> p, cpx<T> v) {
  p->re = v.re;
  p->im = v.im;
}

// Store a piece (aligned to its size) with 16-byte writes, or with one pair
// write per row when it is shorter.
template <typename TM, int ROWS>
__device__ __forceinline__ void store_piece(gptr<TM> dst, const RowPiece<TM, ROWS>& p) {
  constexpr int V = 16 / (int)sizeof(TM);
  if constexpr (2 * ROWS >= V) {
    typedef TM vec_t __attribute__((ext_vector_type(V)));
    const auto d = reinterpret_cast<gptr<vec_t>>(dst);
#pragma unroll
    for (int c = 0; c < 2 * ROWS / V; ++c) {
      vec_t v;
#pragma unroll
      for (int e = 0; e < V; ++e) v[e] = p.v[c * V + e];
      d[c] = v;
    }
  } else {
    typedef TM pair_t __attribute__((ext_vector_type(2)));
    const auto d = reinterpret_cast<gptr<pair_t>>(dst);
#pragma unroll
    for (int r = 0; r < ROWS; ++r) d[r] = pair_t{p.v[2 * r], p.v[2 * r + 1]};
  }
}

// Load a piece (aligned to its size) with 16-byte reads, or with one pair
// read when it is shorter.
template <typename TM, int ROWS>
__device__ __forceinline__ void load_piece(gptr<const TM> src, RowPiece<TM, ROWS>& p) {
  constexpr int V = 16 / (int)sizeof(TM);
  constexpr int W = 2 * ROWS >= V ? V : 2;
  typedef TM vec_t __attribute__((ext_vector_type(W)));
  const auto s = reinterpret_cast<gptr<const vec_t>>(src);
#pragma unroll
  for (int c = 0; c < 2 * ROWS / W; ++c) {
    const vec_t v = s[c];
#pragma unroll
    for (int e = 0; e < W; ++e) p.v[c * W + e] = v[e];
  }
}

// P1b: orthonormal DCT-II along x of the eight row-major fields, for a band
// of ROWS rows, into the strip-major intermediates.
// Each round of the row pass loads NP field pairs of its ROWS rows into LDS
// lines (row r, pair l at (r NP + l) NX, two real fields per complex line) and
// transforms them with one batched FFT; 4 / NP rounds cover the pairs.
template <typename TM, int NX, int V>
using RowDctLds = LinesLds<TM, p1_rows_v<TM>(NX, V) * p1_pairs_v<TM>(NX, V) * NX, NX>;

template <typename TM, int NX, int V>
__device__ __forceinline__ void row_dct8_body(gptr<const TM> __restrict__ rm,
                                              gptr<TM> __restrict__ mid,
                                              int ny, int blk, RowDctLds<TM, NX, V>& L, int tid) {
  constexpr int NTHR = line_threads(NX);
  constexpr int ROWS = p1_rows_v<TM>(NX, V);
  constexpr int NP = p1_pairs_v<TM>(NX, V);
  cpx<TM>* line = L.line;
  cpx<double>* rtab = L.rtab;
  const int j0 = blk * ROWS;
  const size_t FS = (size_t)NX * ny;                            // row-major fields
  const size_t SS = strip_stride(ny, sizeof(TM));
  const size_t FSM = strip_field(NX, ny, sizeof(TM));           // strip-major fields
  const size_t SSP = pair_strip_stride(ny), FSP = pair_field(NX, ny);   // FP32 pairs
  Roots<TM, NX> rt;
  rt.init(rtab, tid, NTHR);

  using MAP = LdsMap<TM, NX, SWZ_ROW>;
  constexpr int R = fft_radix<TM>();
  using LS = LineSlots<NX, NTHR, R, MAP>;
  constexpr int CPT = NX >= NTHR ? NX / NTHR : 1;            // loads per thread and line
  // Post-processing: HALVES lanes share the rows of one column pair sp, so
  // that the band's values of a field (FP64) or of a field pair (FP32, both
  // fields side by side in each row) leave as one piece of ROWS x 16 bytes,
  // written by adjacent lanes in the same store instruction (lane h of the
  // pair takes rows h RH .. h RH + RH - 1).
  constexpr int HALVES = ROWS >= 2 ? 2 : 1;
  constexpr int RH = ROWS / HALVES;
  constexpr int SPL = NTHR / HALVES;                         // column pairs per pass
  constexpr int SPT = NX / 2 >= SPL ? NX / 2 / SPL : 1;      // passes
  const TM S0 = (TM)(0.5 * sqrt(1.0 / NX)), S1 = (TM)(0.5 * sqrt(2.0 / NX));

  auto round = [&](auto ir) {
    constexpr int r = decltype(ir)::value;
    // Each round forms its LDS slots (a per-thread base XOR a constant) from
    // a thread index of its own, so that the compiler does not hold them
    // from round to round (at the register cap it spilled them).
    const int tt = opaque_vgpr(tid);
    const LS sl(tt);
    const int spt = tt / HALVES, half = tt % HALVES;
    // Slots of bins 2 sp and 2 sp + 1 and of their mirrors
    // N - 2 sp = (N - 1) ^ (2 (sp - 1) + 1) and N - 2 sp - 1 = (N - 1) ^ 2 sp,
    // for sp = spt + it SPL (2 sp = 2 spt + it 2 SPL, disjoint bits).
    const int g2 = LS::g(2 * spt);
    const int g2m = MAP::at(NX - 1) ^ LS::g(1) ^ LS::g((2 * spt - 2) & (NX - 1));
#pragma unroll
    for (int rr = 0; rr < ROWS; ++rr) {
#pragma unroll
      for (int l = 0; l < NP; ++l) {
        const int pr = r * NP + l;
        const auto ra = rm + RowPairs<TM>::A[pr] * FS + (size_t)(j0 + rr) * NX;
        const auto rb = rm + RowPairs<TM>::B[pr] * FS + (size_t)(j0 + rr) * NX;
        const int lo = MAP::at((rr * NP + l) * NX);
        static_for<CPT>([&](auto iq) {
          constexpr int q = decltype(iq)::value;
          const int i = tt + q * NTHR;
          if (NX >= NTHR || i < NX) line[lo ^ sl.template mak<q>()] = {ra[i], rb[i]};
        });
      }
    }
    lds_sync();
    fft_lines<TM, NX, ROWS * NP, NTHR, R, MAP>(line, rt, tt);
#pragma unroll 1
    for (int it = 0; it < SPT; ++it) {
      const int sp = spt + it * SPL;
      if (NX / 2 >= SPL || sp < NX / 2) {
        const int pk0 = g2 ^ LS::g(2 * it * SPL);
        const int pk1 = pk0 ^ LS::g(1);
        const int pm1 = pk0 ^ MAP::at(NX - 1);
        const int pm0 = spt == 0 ? (it == 0 ? 0 : (MAP::at(NX - 1) ^ LS::g(1) ^
                                                   LS::g((2 * it * SPL - 2) & (NX - 1))))
                                 : (g2m ^ LS::g(2 * it * SPL));
        const cpx<TM> w0 = rt.omega(2 * sp), w1 = rt.omega(2 * sp + 1);
        const TM s0 = sp == 0 ? S0 : S1;
#pragma unroll
        for (int l = 0; l < NP; ++l) {
          const int pr = r * NP + l;
          RowPiece<TM, RH> pa, pb;
#pragma unroll
          for (int q = 0; q < RH; ++q) {
            const int rr = half * RH + q;
            const int lo = MAP::at((rr * NP + l) * NX);
            dct2_bin<TM>(line[lo ^ pk0], line[lo ^ pm0], w0, s0, pa.v[2 * q], pb.v[2 * q]);
            dct2_bin<TM>(line[lo ^ pk1], line[lo ^ pm1], w1, S1, pa.v[2 * q + 1],
                         pb.v[2 * q + 1]);
          }
          if constexpr (sizeof(TM) == 4) {
            // both fields' rows, interleaved, as one piece
            RowPiece<TM, 2 * RH> pc;
#pragma unroll
            for (int q = 0; q < RH; ++q) {
              pc.v[4 * q] = pa.v[2 * q];
              pc.v[4 * q + 1] = pa.v[2 * q + 1];
              pc.v[4 * q + 2] = pb.v[2 * q];
              pc.v[4 * q + 3] = pb.v[2 * q + 1];
            }
            const size_t o = (size_t)sp * SSP + 4 * (size_t)(j0 + half * RH);
            store_piece<TM, 2 * RH>(mid + mid_pair(RowPairs<TM>::A[pr]) * FSP + o, pc);
          } else {
            const size_t o = (size_t)sp * SS + 2 * (size_t)(j0 + half * RH);
            store_piece<TM, RH>(mid + RowPairs<TM>::A[pr] * FSM + o, pa);
            store_piece<TM, RH>(mid + RowPairs<TM>::B[pr] * FSM + o, pb);
          }
        }
      }
    }
    lds_sync();
  };
  round(std::integral_constant<int, 0>{});
  if constexpr (NP <= 2) round(std::integral_constant<int, 1>{});
  if constexpr (NP == 1) {
    round(std::integral_constant<int, 2>{});
    round(std::integral_constant<int, 3>{});
  }
}

// ---------------------------------------------------------------------------
// P2: column DCT-II of the eight fields and the spectral Gram sums.
// ---------------------------------------------------------------------------
// One strip (two columns of one field) held in registers, LPT elements per
// thread (natural index tid + q NTHR).
template <typename TM, int LPT> struct StripRegs {
  cpx<TM> v[LPT];
};

// Row jj of the strip is src[jj STRIDE] (STRIDE 2: one field of an FP32 pair
// region, the other field's values in between).
template <typename TM, int NY, int LPT, int NTHR, int STRIDE = 1>
__device__ __forceinline__ void fetch_strip(gptr<const cpx<TM>> __restrict__ src, int tid,
                                            StripRegs<TM, LPT>& r) {
#pragma unroll
  for (int q = 0; q < LPT; ++q) {
    const int jj = tid + q * NTHR;
    r.v[q] = (NY >= NTHR || jj < NY) ? gload<TM>(src + jj * STRIDE) : cpx<TM>{(TM)0, (TM)0};
  }
}

// Both fields of a strip of an FP32 pair region (mid_pair), the thread's
// rows q = Q0 .. Q1 - 1: row jj is one 16-byte load; a takes the first field,
// b the second.
template <typename TM, int NY, int LPT, int NTHR, int Q0, int Q1>
__device__ __forceinline__ void fetch_pair_strip(gptr<const TM> __restrict__ src, int tid,
                                                 StripRegs<TM, LPT>& a, StripRegs<TM, LPT>& b) {
  typedef TM tm4 __attribute__((ext_vector_type(4)));
  const auto p = reinterpret_cast<gptr<const tm4>>(src);
#pragma unroll
  for (int q = Q0; q < Q1; ++q) {
    const int jj = tid + q * NTHR;
    const tm4 v = (NY >= NTHR || jj < NY) ? p[jj] : tm4{(TM)0, (TM)0, (TM)0, (TM)0};
    a.v[q] = {v[0], v[1]};
    b.v[q] = {v[2], v[3]};
  }
}

// Whether the column transform can take its first FFT stage straight from the
// loaded registers: one radix-R butterfly per thread in every stage, so that
// thread tid's first butterfly reads Makhoul-ordered elements tid + q (N/R).
template <int NY, int NTHR, int R> constexpr bool first_stage_in_registers() {
  return NY / R == NTHR && Plan<NY, R>::FIRST == R && NY > R;
}

// Loads for first_stage_in_registers: v[q] = element k = tid + q (NY/R) of the
// Makhoul-reordered strip, i.e. row 2k for k < NY/2 and row 2(NY-1-k)+1 above.
template <typename TM, int NY, int R, int NTHR, int STRIDE = 1>
__device__ __forceinline__ void fetch_strip_first(gptr<const cpx<TM>> __restrict__ src, int tid,
                                                  StripRegs<TM, R>& r) {
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int k = tid + q * (NY / R);
    const int row = k < NY / 2 ? 2 * k : 2 * (NY - 1 - k) + 1;
    r.v[q] = gload<TM>(src + row * STRIDE);
  }
}

// fetch_strip_first for both fields of an FP32 pair strip, rows q = Q0 .. Q1 - 1.
template <typename TM, int NY, int R, int NTHR, int Q0, int Q1>
__device__ __forceinline__ void fetch_pair_strip_first(gptr<const TM> __restrict__ src, int tid,
                                                       StripRegs<TM, R>& a, StripRegs<TM, R>& b) {
  typedef TM tm4 __attribute__((ext_vector_type(4)));
  const auto p = reinterpret_cast<gptr<const tm4>>(src);
#pragma unroll
  for (int q = Q0; q < Q1; ++q) {
    const int k = tid + q * (NY / R);
    const int row = k < NY / 2 ? 2 * k : 2 * (NY - 1 - k) + 1;
    const tm4 v = p[row];
    a.v[q] = {v[0], v[1]};
    b.v[q] = {v[2], v[3]};
  }
}

// DCT-II along y of a strip held in registers: A (column 2s) and B (column
// 2s + 1) for the bins of the thread's pair units u = tid + q NTHR, bin u at
// index 2q and bin pair_mirror(u) at 2q + 1. The FFT radix R gives one
// butterfly per thread in each stage. With FIRST_IN_REGS the registers hold
// the inputs of the thread's first-stage butterfly (fetch_strip_first): that
// stage runs on them and stores its outputs, saving one pass through LDS.
// TRAIL_SYNC false: the caller writes its next line elsewhere, so the last
// reads of this one need no barrier behind them.
template <typename TM, int NY, int LPT, int UPT, int NTHR, int R, typename MAP,
          bool FIRST_IN_REGS = false, bool TRAIL_SYNC = true>
__device__ __forceinline__ void column_dct2(const StripRegs<TM, LPT>& in, cpx<TM>* line,
                                            const Roots<TM, NY>& rt,
                                            const LineSlots<NY, NTHR, R, MAP>& sl, int tid,
                                            TM (&A)[2 * UPT], TM (&B)[2 * UPT]) {
  if constexpr (FIRST_IN_REGS) {
    static_assert(LPT == R && first_stage_in_registers<NY, NTHR, R>(), "one butterfly per thread");
    // the first stage of fft_lines (block length NY, stride NY/R) on butterfly tid
    constexpr int S = NY / R;
    cpx<TM> v[R];
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = in.v[q];
    SmallDFT<TM, R>::run(v);
    apply_twiddles<TM, NY, R>(rt, tid, v);
    const int e = MAP::at(tid);
#pragma unroll
    for (int q = 0; q < R; ++q) line[e ^ MAP::at(q * S)] = v[q];
    lds_sync();
    DifRunner<TM, NY, 1, NTHR, S, false, R, MAP>::run(line, rt, tid);
  } else {
    static_for<LPT>([&](auto iq) {
      constexpr int q = decltype(iq)::value;
      if (NY >= NTHR || tid + q * NTHR < NY) line[sl.template mak<q>()] = in.v[q];
    });
    lds_sync();
    fft_lines<TM, NY, 1, NTHR, R, MAP>(line, rt, tid);
  }
  static_for<UPT>([&](auto iq) {
    constexpr int q = decltype(iq)::value;
    const int u = tid + q * NTHR;
    if (NY / 2 >= NTHR || u < NY / 2) {
      dct2_unit<TM, NY>(line, sl.template bin<q>(), sl.template binm<q>(), rt, u, A[2 * q],
                        B[2 * q], A[2 * q + 1], B[2 * q + 1]);
    } else {
      A[2 * q] = 0; B[2 * q] = 0; A[2 * q + 1] = 0; B[2 * q + 1] = 0;
    }
  });
  if constexpr (TRAIL_SYNC) lds_sync();
}

// Sum NV per-thread values over the block and add them to acc[IDX[q]].
template <int NV, int NTHR>
__device__ __forceinline__ void stage_accumulate(double (&v)[NV], const int (&idx)[NV],
                                                 double* red, double* acc, int tid) {
  block_sum<NV, NTHR>(v, red, tid);
  if (tid < NV) acc[idx[tid]] += red[tid];
}

// LDS plan of the Gram kernel: the line, the S~ spectrum (waiting for its
// products with the later fields) and, where they fit, per-thread partial
// sums that are reduced over the block once per strip instead of once per
// field.
template <typename TM, int NY> struct GramPlan {
  static constexpr int NTHR = gram_threads<TM>(NY);
  static constexpr int LINE_B = NY * (int)sizeof(cpx<TM>);
  static constexpr int ROOT_B = Roots<TM, NY>::SIZE * (int)sizeof(cpx<double>);
  // The partial sums only go to LDS while the CU still holds 8 waves of
  // workgroups.
  static constexpr int BUDGET = 150 * 1024;
  static constexpr int WAVES = NTHR / 64;
  static constexpr int ACC_BUDGET = WAVES >= 8 ? BUDGET : (160 * 1024) / (8 / WAVES);
  static constexpr int ACC_B = P2_NSUM * NTHR * (int)sizeof(double);
  // FP32 workgroups of 8 waves (one per CU): two line buffers, alternating
  // from field to field, where they fit beside the partial sums (the S~
  // spectrum then stays in registers), so that a transform needs no barrier
  // after its last reads of its line. (With 4 waves the extra registers would
  // halve the waves per SIMD.)
  static constexpr bool DBL = sizeof(TM) == 4 && NTHR == 512 &&
                              2 * LINE_B + ROOT_B + ACC_B <= ACC_BUDGET;
  static constexpr bool S_LDS = !DBL && 2 * LINE_B + ROOT_B <= BUDGET;
  static constexpr bool ACC_LDS =
      (S_LDS || DBL ? 2 : 1) * LINE_B + ROOT_B + ACC_B <= ACC_BUDGET && NTHR % 16 == 0;
  // FP32 lines of 8192 points and more: sixteen bins per thread leave no
  // registers for the kept spectra beside a transform, so they go to
  // per-thread slots in global memory (the stencil output region, unused
  // while this pass runs), written once and read once by the same thread,
  // coalesced across the wave.
  static constexpr bool KEEP_GLOBAL = NY >= 8192;
};
template <typename TM, int NY> struct GramLds {
  using GP = GramPlan<TM, NY>;
  cpx<TM> line[(GP::DBL ? 2 : 1) * NY];
  cpx<TM> keep[GP::S_LDS ? NY : 1];
  cpx<double> rtab[Roots<TM, NY>::SIZE];
  double red[GP::ACC_LDS ? 1 : P2_NSUM * (GP::NTHR / 64 + 1)];   // per-field block sums
  double acc[GP::ACC_LDS ? P2_NSUM * GP::NTHR : P2_NSUM];
};

// FRESH_SLOTS: every transform forms its LDS slots anew (the persistent
// launch, where the kernel's register budget is shared by all passes).
template <typename TM, int NY, bool FRESH_SLOTS = false>
__device__ __forceinline__ void col_gram_body(gptr<const TM> __restrict__ mid,
                                              gptr<const double> __restrict__ lamx,
                                              gptr<const double> __restrict__ lamy,
                                              gptr<double> __restrict__ part, int nx,
                                              const OpConst c, int s, GramLds<TM, NY>& L,
                                              int tid, gptr<TM> __restrict__ kg) {
  using GP = GramPlan<TM, NY>;
  constexpr int NTHR = GP::NTHR;
  constexpr int LPT = NY >= NTHR ? NY / NTHR : 1;            // strip loads per thread
  constexpr int UPT = NY / 2 >= NTHR ? NY / 2 / NTHR : 1;    // pair units per thread
  constexpr int KPT = 2 * UPT;                               // bins per thread
  constexpr int KS = NY / 2 >= NTHR ? NTHR : NY / 2;         // stride of a thread's bins in keep
  // Radix with one butterfly per thread in each FFT stage.
  constexpr int GR = NY / NTHR >= 8 ? 8 : (NY / NTHR >= 4 ? 4 : 2);
  using MAP = LdsMap<TM, NY, SWZ_GRAM>;
  using LS = LineSlots<NY, NTHR, GR, MAP>;
  constexpr bool S_LDS = GP::S_LDS;
  constexpr bool ACC_LDS = GP::ACC_LDS;
  cpx<TM>* line = L.line;
  cpx<TM>* keep = L.keep;
  cpx<double>* rtab = L.rtab;
  double* red = L.red;
  double* acc = L.acc;
  const size_t SS = strip_stride(NY, sizeof(TM));
  const size_t FSM = strip_field(nx, NY, sizeof(TM));
  Roots<TM, NY> rt;
  rt.init(rtab, tid, NTHR);
  const LS sl(tid);
  if constexpr (ACC_LDS) {
#pragma unroll
    for (int q = 0; q < P2_NSUM; ++q) acc[q * NTHR + tid] = 0.0;
  } else {
    if (tid < P2_NSUM) acc[tid] = 0.0;
  }
  // Adds the thread's stage sums v[b] to sum idx[b].
  auto accumulate = [&](auto& v, const auto& idx) {
    constexpr int NV = sizeof(v) / sizeof(double);
    if constexpr (ACC_LDS) {
#pragma unroll
      for (int b = 0; b < NV; ++b) acc[idx[b] * NTHR + tid] += v[b];
    } else {
      stage_accumulate<NV, NTHR>(v, idx, red, acc, tid);
    }
  };
  const double lx0 = lamx[2 * s], lx1 = lamx[2 * s + 1];
  auto strip = [&](int f) {
    return reinterpret_cast<gptr<const cpx<TM>>>(mid + (size_t)f * FSM + (size_t)s * SS);
  };
  // bin held at index j (unit tid + (j / 2) NTHR; even j: the unit's own bin)
  auto bin_of = [&](int j) {
    const int u = tid + (j >> 1) * NTHR;
    return (j & 1) ? pair_mirror<NY>(u) : u;
  };
  const bool valid = NY / 2 >= NTHR || tid < NY / 2;
  // 1/sigma (chi) or 1/tau (zeta) at (2s, k) and (2s+1, k)
  auto inv_op = [&](int k, bool chi, double& i0, double& i1) {
    const double ly = lamy[k];
    const double L0 = lx0 + ly, L1 = lx1 + ly;
    if (chi) {
      i0 = rcp64(c.C1 + L0 * (c.C2 + c.C3 * L0));
      i1 = rcp64(c.C1 + L1 * (c.C2 + c.C3 * L1));
    } else {
      i0 = rcp64(c.alpha + c.lam * L0);
      i1 = rcp64(c.alpha + c.lam * L1);
    }
  };
  // Spectra kept for the pairwise products: index 0 = S~ (unless in LDS),
  // 1 = H, 2 = Q~, 3 = K~; later 1 = P~ and 2 = g_lin. With GP::KEEP_GLOBAL
  // slot f of bin index j is element (f KPT + j) NTHR + tid of this strip's
  // block of 4 NY complex values in kg.
  constexpr bool KG = GP::KEEP_GLOBAL;
  constexpr int KR = KG ? 1 : KPT;
  TM ka[4][KR], kb[4][KR];
  typedef TM tm2 __attribute__((ext_vector_type(2)));
  const auto kgs = reinterpret_cast<gptr<tm2>>(kg) + (size_t)s * 4 * NY + tid;
  auto kept = [&](int f, int j, TM& a, TM& b) {
    if (S_LDS && f == 0) {
      const cpx<TM> v = keep[tid + j * KS];
      a = v.re;
      b = v.im;
    } else if constexpr (KG) {
      const tm2 v = kgs[(f * KPT + j) * NTHR];
      a = v[0];
      b = v[1];
    } else {
      a = ka[f][j];
      b = kb[f][j];
    }
  };
  auto put = [&](int f, int j, TM a, TM b) {
    if constexpr (KG) {
      kgs[(f * KPT + j) * NTHR] = tm2{a, b};
    } else {
      ka[f][j] = a;
      kb[f][j] = b;
    }
  };
  // Fields in the order they are transformed. With FP32 lines the fields
  // come in the pairs of their layout (mid_pair), consecutive in this order:
  // one 16-byte load per row brings a field and the next. The next pair is
  // loaded while the current one is transformed, half of its rows during
  // each of the two transforms. FP64 lines (one field per region) and
  // workgroups of more than 8 waves (at most 128 registers per thread) have
  // no registers to spare for loads ahead: they load each field when it is
  // transformed (FP32: its half of the pair region, the other half read
  // from L2 one transform later).
  constexpr int ORDER[8] = {M_S, M_H, M_Q, M_K, M_F, M_P, M_G, M_L};
  static_assert(mid_pair(ORDER[0]) == mid_pair(ORDER[1]) && mid_half(ORDER[0]) == 0 &&
                    mid_pair(ORDER[2]) == mid_pair(ORDER[3]) && mid_half(ORDER[2]) == 0 &&
                    mid_pair(ORDER[4]) == mid_pair(ORDER[5]) && mid_half(ORDER[4]) == 0 &&
                    mid_pair(ORDER[6]) == mid_pair(ORDER[7]) && mid_half(ORDER[6]) == 0,
                "the transform order takes the pairs' fields one after the other");
  constexpr bool PAIRS = sizeof(TM) == 4 && NTHR <= 512 && !GP::KEEP_GLOBAL;
  // The first FFT stage runs on the loaded registers where every stage has
  // one butterfly per thread.
  constexpr bool FIRST_IN_REGS = first_stage_in_registers<NY, NTHR, GR>() && LPT == GR;
  auto fetch = [&](int f, StripRegs<TM, LPT>& r) {
    if constexpr (FIRST_IN_REGS) {
      fetch_strip_first<TM, NY, GR, NTHR>(strip(f), tid, r);
    } else {
      fetch_strip<TM, NY, LPT, NTHR>(strip(f), tid, r);
    }
  };
  // FP32: the fields of pair k in set k % 2
  StripRegs<TM, LPT> pa[2], pb[2];
  constexpr int QH = LPT >= 2 ? LPT / 2 : LPT;
  auto fetch_pair = [&](int f, auto iset, auto iq0, auto iq1) {
    constexpr int st = decltype(iset)::value, q0 = decltype(iq0)::value,
                  q1 = decltype(iq1)::value;
    const auto src = mid + mid_pair(f) * pair_field(nx, NY) + (size_t)s * pair_strip_stride(NY);
    if constexpr (FIRST_IN_REGS) {
      fetch_pair_strip_first<TM, NY, GR, NTHR, q0, q1>(src, tid, pa[st], pb[st]);
    } else {
      fetch_pair_strip<TM, NY, LPT, NTHR, q0, q1>(src, tid, pa[st], pb[st]);
    }
  };
  using I0 = std::integral_constant<int, 0>;
  using IH = std::integral_constant<int, QH>;
  using IL = std::integral_constant<int, LPT>;
  if constexpr (PAIRS) fetch_pair(ORDER[0], I0{}, I0{}, IL{});
  // FP32 lines with the kept spectra in global memory: a pair's strip is
  // loaded once, with 16-byte loads, when its first field is transformed;
  // the second field waits in registers (loading each half on its own
  // fetched the pair's sectors twice).
  constexpr bool KG_PAIR = GP::KEEP_GLOBAL && sizeof(TM) == 4;
  StripRegs<TM, KG_PAIR ? LPT : 1> kg_second;
  auto transform_next = [&](auto ii, TM (&A)[KPT], TM (&B)[KPT]) {
    constexpr int i = decltype(ii)::value;
    StripRegs<TM, LPT> cur;
    if constexpr (PAIRS) {
      constexpr int cs = (i / 2) % 2, ns = 1 - cs;
      using INS = std::integral_constant<int, ns>;
      if constexpr (i % 2 == 0) {
        cur = pa[cs];
        if constexpr (i + 2 < 8) fetch_pair(ORDER[i + 2], INS{}, I0{}, IH{});
      } else {
        cur = pb[cs];
        if constexpr (i + 1 < 8 && QH < LPT) fetch_pair(ORDER[i + 1], INS{}, IH{}, IL{});
      }
    } else if constexpr (GP::KEEP_GLOBAL) {
      // The eight transforms form their LDS slots (a per-thread base XOR a
      // constant) from a thread index of their own, so that the compiler
      // does not hold each slot across the kernel (it spilled them).
      static_assert(!GP::DBL && !FIRST_IN_REGS, "one line buffer, loads into LDS");
      const int tt = opaque_vgpr(tid);
      const LS slt(tt);
      if constexpr (KG_PAIR) {
        if constexpr (i % 2 == 0) {
          const auto src =
              mid + mid_pair(ORDER[i]) * pair_field(nx, NY) + (size_t)s * pair_strip_stride(NY);
          fetch_pair_strip<TM, NY, LPT, NTHR, 0, LPT>(src, tt, cur, kg_second);
        } else {
          cur = kg_second;
        }
      } else {
        fetch_strip<TM, NY, LPT, NTHR>(strip(ORDER[i]), tt, cur);
      }
      column_dct2<TM, NY, LPT, UPT, NTHR, GR, MAP, false, true>(cur, line, rt, slt, tt, A, B);
      return;
    } else if constexpr (sizeof(TM) == 4) {
      const auto src = reinterpret_cast<gptr<const cpx<TM>>>(
          mid + mid_pair(ORDER[i]) * pair_field(nx, NY) + (size_t)s * pair_strip_stride(NY) +
          2 * mid_half(ORDER[i]));
      if constexpr (FIRST_IN_REGS) {
        fetch_strip_first<TM, NY, GR, NTHR, 2>(src, tid, cur);
      } else {
        fetch_strip<TM, NY, LPT, NTHR, 2>(src, tid, cur);
      }
    } else {
      fetch(ORDER[i], cur);
    }
    // field i's line (alternating buffers where GP::DBL)
    cpx<TM>* ln = GP::DBL ? line + (i % 2) * NY : line;
    if constexpr (sizeof(TM) == 8 || FRESH_SLOTS) {
      // FP64 lines form their slots per transform as well: fewer registers
      // held across the kernel, two workgroups per CU at N = 1024 and 2048
      // (with FP32 lines in their own launch the extra address arithmetic
      // costs more than the registers it frees).
      const int tt = opaque_vgpr(tid);
      const LS slt(tt);
      column_dct2<TM, NY, LPT, UPT, NTHR, GR, MAP, FIRST_IN_REGS, !GP::DBL>(cur, ln, rt, slt, tt,
                                                                          A, B);
    } else {
      column_dct2<TM, NY, LPT, UPT, NTHR, GR, MAP, FIRST_IN_REGS, !GP::DBL>(cur, ln, rt, sl, tid,
                                                                          A, B);
    }
  };
  // chi group: S~, H, Q~, K~ transformed and kept; their inner products are
  // taken together with those of f_lin, bin by bin, so that each bin's
  // weights 1/sigma are formed once.
  auto keep_stage = [&](auto ia) {
    constexpr int a = decltype(ia)::value;
    TM A[KPT], B[KPT];
    transform_next(ia, A, B);
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
      if (S_LDS && a == 0) {
        if (valid) keep[tid + j * KS] = {A[j], B[j]};
      } else {
        put(a, j, A[j], B[j]);
      }
    }
  };
  keep_stage(std::integral_constant<int, 0>{});
  keep_stage(std::integral_constant<int, 1>{});
  keep_stage(std::integral_constant<int, 2>{});
  keep_stage(std::integral_constant<int, 3>{});
  {
    TM A[KPT], B[KPT];
    transform_next(std::integral_constant<int, 4>{}, A, B);
    // pairs (x, y) of {S~, H, Q~, K~, f_lin} = indices 0..4
    constexpr int NPR = 14;
    constexpr int PX[NPR] = {0, 0, 0, 0, 1, 1, 1, 2, 2, 3, 4, 4, 4, 4};
    constexpr int PY[NPR] = {0, 1, 2, 3, 1, 2, 3, 2, 3, 3, 0, 1, 2, 3};
    const int idx[NPR] = {P2_SS, P2_SH, P2_SQ, P2_SK, P2_HH, P2_HQ, P2_HK,
                          P2_QQ, P2_QK, P2_KK, P2_FS, P2_FH, P2_FQ, P2_FK};
    double v[NPR];
#pragma unroll
    for (int q = 0; q < NPR; ++q) v[q] = 0.0;
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
      if (!valid) continue;                  // blocks wider than half the line
      double i0, i1;
      inv_op(bin_of(j), true, i0, i1);
      double xa[5], xb[5];
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        TM ea, eb;
        kept(f, j, ea, eb);
        xa[f] = (double)ea;
        xb[f] = (double)eb;
      }
      xa[4] = (double)A[j];
      xb[4] = (double)B[j];
      double wa[5], wb[5];
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        wa[f] = xa[f] * i0;
        wb[f] = xb[f] * i1;
      }
#pragma unroll
      for (int q = 0; q < NPR; ++q) v[q] += wa[PX[q]] * xa[PY[q]] + wb[PX[q]] * xb[PY[q]];
      __builtin_amdgcn_sched_barrier(0);
    }
    accumulate(v, idx);
  }
  // zeta group: P~ and g_lin kept (in the H and Q~ slots), then L~; both
  // inner products with one weight per bin.
  if constexpr (KG) {
    auto keep_zeta = [&](auto ii, int f) {
      TM A[KPT], B[KPT];
      transform_next(ii, A, B);
#pragma unroll
      for (int j = 0; j < KPT; ++j) put(f, j, A[j], B[j]);
    };
    keep_zeta(std::integral_constant<int, 5>{}, 1);
    keep_zeta(std::integral_constant<int, 6>{}, 2);
  } else {
    transform_next(std::integral_constant<int, 5>{}, ka[1], kb[1]);
    transform_next(std::integral_constant<int, 6>{}, ka[2], kb[2]);
  }
  {
    TM A[KPT], B[KPT];
    transform_next(std::integral_constant<int, 7>{}, A, B);
    double v[2] = {0.0, 0.0};
    const int idx[2] = {P2_PG, P2_PL};
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
      if (!valid) continue;
      double i0, i1;
      inv_op(bin_of(j), false, i0, i1);
      TM p0, p1, g0, g1;
      kept(1, j, p0, p1);
      kept(2, j, g0, g1);
      const double pa = (double)p0 * i0, pb = (double)p1 * i1;
      v[0] += pa * (double)g0 + pb * (double)g1;
      v[1] += pa * (double)A[j] + pb * (double)B[j];
    }
    accumulate(v, idx);
  }
  if constexpr (ACC_LDS) {
    // Sum the per-thread partials: thread t adds 16 consecutive threads'
    // values of sum t / (NTHR / 16) (in a rotated order that keeps the lanes
    // on different banks), then 16 threads add the chunks.
    constexpr int CH = NTHR / 16;
    lds_sync();
    const int q = tid / CH, ch = tid % CH;
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) t += acc[q * NTHR + 16 * ch + ((i + ch) & 15)];
    lds_sync();
    acc[q * NTHR + ch] = t;
    lds_sync();
    if (tid < P2_NSUM) {
      double u = 0.0;
      for (int i = 0; i < CH; ++i) u += acc[tid * NTHR + i];
      part[(size_t)s * P2_NSUM + tid] = u;
    }
  } else {
    lds_sync();
    if (tid < P2_NSUM) part[(size_t)s * P2_NSUM + tid] = acc[tid];
  }
}

// ---------------------------------------------------------------------------
// Reduction helpers shared by the single-workgroup kernels.
// ---------------------------------------------------------------------------
template <int NV, int NTHR, typename P>
__device__ void reduce_rows(P part, int nrows, double* red, int tid, double (&tot)[NV]) {
  double v[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = 0.0;
  for (int r = tid; r < nrows; r += NTHR) {
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] += part[(size_t)r * NV + q];
  }
  block_sum<NV, NTHR>(v, red, tid);
#pragma unroll
  for (int q = 0; q < NV; ++q) tot[q] = red[q];
  lds_sync();
}

// Column sums of an nrows x NV row-major array of partials. Thread t < G NV
// (G = NTHR / NV row groups) adds column t mod NV over rows t / NV + i G, so a
// wave's loads read consecutive doubles; the G group sums of a column are then
// added in group order, a fixed order for any launch. Every thread receives
// the totals; red holds NTHR + NV doubles.
template <int NV, int NTHR, typename P>
__device__ void reduce_columns(P part, int nrows, double* red, int tid, double (&tot)[NV]) {
  static_assert(NV <= NTHR, "one thread per column at least");
  constexpr int G = NTHR / NV;
  constexpr size_t ACT = (size_t)G * NV;
  // The kernel is bound by load latency: every round issues U independent
  // loads per thread (absent ones read as zero) before adding them in order.
  constexpr int U = 16;
  const size_t total = (size_t)nrows * NV;
  double v = 0.0;
  if ((size_t)tid < ACT) {
    for (size_t e = tid; e < total; e += U * ACT) {
      double a[U];
#pragma unroll
      for (int u = 0; u < U; ++u) a[u] = e + u * ACT < total ? part[e + u * ACT] : 0.0;
#pragma unroll
      for (int u = 0; u < U; ++u) v += a[u];
    }
  }
  red[tid] = v;
  lds_sync();
  if (tid < NV) {
    double t = 0.0;
    for (int g = 0; g < G; ++g) t += red[g * NV + tid];
    red[NTHR + tid] = t;
  }
  lds_sync();
#pragma unroll
  for (int q = 0; q < NV; ++q) tot[q] = red[NTHR + q];
  lds_sync();
}

// ---------------------------------------------------------------------------
// S: the 5x5 reduced system of App. B, Step 4, and the SAV update.
// ---------------------------------------------------------------------------
// Threads of the 5x5 kernel: 512 for grids above 512^2 (thousands of partial
// rows, read with many loads in flight), 256 up to 512^2. The two orders of
// the partial sums differ, so every path of one grid uses the same count.
constexpr int SOLVE_THREADS = 512;
constexpr int SOLVE_THREADS_SMALL = 256;
inline int solve_threads(size_t cells) {
  return cells > (size_t)512 * 512 ? SOLVE_THREADS : SOLVE_THREADS_SMALL;
}
constexpr int SOLVE_NV_MAX = (int)P1_NSUM > (int)P2_NSUM ? (int)P1_NSUM : (int)P2_NSUM;
template <int NTHR> struct SolveLds {
  double red[NTHR + SOLVE_NV_MAX];
};

// The 5x5 system from the reduced sums T1 (stencil pass) and T2 (column
// pass), its solution, the new SAVs and the combination coefficients; run by
// one thread.
__device__ __forceinline__ void solve_system(const double (&T1)[P1_NSUM], double (&T2)[P2_NSUM],
                                             gptr<DevScalars> __restrict__ ds,
                                             const StepConst& c) {
  int err = 0;
  const double h2 = c.h2;
  const double rS2 = h2 * T1[P1_RS], rW2 = h2 * T1[P1_RW], rZ2 = h2 * T1[P1_RZ];
  const double tiny = 1e-280;
  if (!(rS2 > tiny) || !(rW2 > tiny) || !(rZ2 > tiny)) err |= ERR_NORM;
  const double nS = 1.0 / sqrt(rS2), nQ = 1.0 / sqrt(rW2), nK = 1.0 / sqrt(rZ2);
  const double nF[4] = {nS, 1.0, nQ, nK};
  const auto Vn = ds->sav[c.slot_n];
  const auto Vm = ds->sav[c.slot_m];
  double s[4];
  for (int i = 0; i < 4; ++i) s[i] = c.c0 * Vn[i] + c.c1 * Vm[i] + h2 * nF[i] * T1[P1_ES + i];
  s[3] += h2 * nK * T1[P1_EP];

  const int gi[4][4] = {{P2_SS, P2_SH, P2_SQ, P2_SK},
                        {P2_SH, P2_HH, P2_HQ, P2_HK},
                        {P2_SQ, P2_HQ, P2_QQ, P2_QK},
                        {P2_SK, P2_HK, P2_QK, P2_KK}};
  double G[4][4];
  for (int i = 0; i < 4; ++i)
    for (int jx = 0; jx < 4; ++jx) G[i][jx] = h2 * nF[i] * nF[jx] * T2[gi[i][jx]];
  const double cw[4] = {c.cgs, c.cga, c.cgb, c.cgo};
  double M[5][5], b[5];
  for (int i = 0; i < 4; ++i) {
    // (F_i, phi^n) is zero except in the increment form, where the solved
    // right-hand side is chi^{-1} f - phi^n.
    double bi = h2 * nF[i] * (T2[P2_FS + i] + T1[P1_XS + i]);
    for (int jx = 0; jx < 4; ++jx) {
      M[i][jx] = (i == jx ? 1.0 : 0.0) + cw[jx] * G[i][jx];
      bi -= cw[jx] * s[jx] * G[i][jx];
    }
    M[i][4] = c.cgo * G[i][3];
    b[i] = bi;
  }
  if (c.classical) {
    // the classical scheme's zeta is not diagonal in the DCT basis: its two
    // inner products come from the iterative solves, in physical space
    T2[P2_PG] = ds->cl[0];
    T2[P2_PL] = ds->cl[1];
  }
  const double PL = h2 * nK * nK * T2[P2_PL];
  M[4][0] = M[4][1] = M[4][2] = 0.0;
  M[4][3] = -PL;
  M[4][4] = 1.0 - PL;
  b[4] = h2 * nK * (T2[P2_PG] + T1[P1_XP]) + s[3] * PL;
  for (int i = 0; i < 5; ++i) {
    for (int jx = 0; jx < 5; ++jx) ds->diag[15 + 5 * i + jx] = M[i][jx];
  }

  // Gaussian elimination with partial pivoting. Every array index is a
  // compile-time constant (the pivot row is exchanged by selects), so the
  // system stays in registers instead of per-lane scratch memory.
  double scale = 0.0;
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int jx = 0; jx < 5; ++jx) scale = fmax(scale, fabs(M[i][jx]));
#pragma unroll
  for (int col = 0; col < 5; ++col) {
    int piv = col;
    double best = fabs(M[col][col]);
#pragma unroll
    for (int r = col + 1; r < 5; ++r) {
      const double a = fabs(M[r][col]);
      if (a > best) { best = a; piv = r; }
    }
    if (!(best > 1e-14 * scale)) err |= ERR_PIVOT;
#pragma unroll
    for (int r = col + 1; r < 5; ++r) {
      const bool sw = r == piv;
#pragma unroll
      for (int jx = col; jx < 5; ++jx) {
        const double u = M[col][jx], w = M[r][jx];
        M[col][jx] = sw ? w : u;
        M[r][jx] = sw ? u : w;
      }
      const double u = b[col], w = b[r];
      b[col] = sw ? w : u;
      b[r] = sw ? u : w;
    }
#pragma unroll
    for (int r = col + 1; r < 5; ++r) {
      const double m = M[r][col] / M[col][col];
#pragma unroll
      for (int jx = col; jx < 5; ++jx) M[r][jx] -= m * M[col][jx];
      b[r] -= m * b[col];
    }
  }
  double x[5];
#pragma unroll
  for (int r = 4; r >= 0; --r) {
    double t = b[r];
#pragma unroll
    for (int jx = r + 1; jx < 5; ++jx) t -= M[r][jx] * x[jx];
    x[r] = t / M[r][r];
  }
  const double Vnew[4] = {x[0] + s[0], x[1] + s[1], x[2] + s[2], x[3] + x[4] + s[3]};
  const auto coef = ds->coef;
  coef[0] = 1.0;
  coef[1] = -c.cgs * Vnew[0] * nS;
  coef[2] = -c.cga * Vnew[1];
  coef[3] = -c.cgb * Vnew[2] * nQ;
  coef[4] = -c.cgo * Vnew[3] * nK;
  coef[5] = 1.0;
  coef[6] = Vnew[3] * nK;
  coef[7] = 0.0;
  bool finite = true;
  for (int i = 0; i < 4; ++i) {
    ds->sav[c.slot_new][i] = Vnew[i];
    finite = finite && isfinite(Vnew[i]);
    ds->diag[i] = s[i];
  }
  for (int i = 0; i < 5; ++i) ds->diag[7 + i] = x[i];
  ds->diag[4] = sqrt(rS2);
  ds->diag[5] = sqrt(rW2);
  ds->diag[6] = sqrt(rZ2);
  for (int i = 0; i < 7; ++i) finite = finite && isfinite(coef[i]);
  if (!finite) err |= ERR_NONFINITE;
  if (T1[P1_MOBNEG] > 0.0) err |= ERR_MOBILITY;
  if (c.lag_d) ds->acc += c.half_dt * c.lam * c.lam * h2 * T1[P1_DLAG];
  ds->err |= err;
}

// One workgroup reduces all partial rows and solves.
template <int NTHR>
__device__ __forceinline__ void solve_body(gptr<const double> __restrict__ p1, int n1,
                                           gptr<const double> __restrict__ p2, int n2,
                                           gptr<DevScalars> __restrict__ ds, const StepConst& c,
                                           SolveLds<NTHR>& L, int tid) {
  double* red = L.red;
  double T1[P1_NSUM], T2[P2_NSUM];
  reduce_columns<P1_NSUM, NTHR>(p1, n1, red, tid, T1);
  reduce_columns<P2_NSUM, NTHR>(p2, n2, red, tid, T2);
  if (tid == 0) solve_system(T1, T2, ds, c);
}

// SOLVE_SLICES workgroups per grid: workgroup g reduces slice g of the
// partial rows (rows g n / SOLVE_SLICES up to the next slice) into
// ds->slice[g]; the workgroup that finishes last (an agent-scope counter)
// adds the slices in slice order, solves, and sets the counter back to zero
// for the next step. The sums do not depend on which workgroup finishes
// last, so results repeat bit for bit. Workgroup g's slice and its counter
// increment are ordered by a release fence, the last workgroup's reads by an
// acquire fence.
template <int NTHR>
__device__ __forceinline__ void solve_sliced_body(gptr<const double> __restrict__ p1, int n1,
                                                  gptr<const double> __restrict__ p2, int n2,
                                                  gptr<DevScalars> __restrict__ ds,
                                                  const StepConst& c, int g, SolveLds<NTHR>& L,
                                                  int tid) {
  static_assert(NTHR >= P1_NSUM + P2_NSUM, "one thread per sum for the slice totals");
  double* red = L.red;
  __shared__ int last;
  {
    const int a1 = (int)((long long)n1 * g / SOLVE_SLICES);
    const int b1 = (int)((long long)n1 * (g + 1) / SOLVE_SLICES);
    const int a2 = (int)((long long)n2 * g / SOLVE_SLICES);
    const int b2 = (int)((long long)n2 * (g + 1) / SOLVE_SLICES);
    double T1[P1_NSUM], T2[P2_NSUM];
    reduce_columns<P1_NSUM, NTHR>(p1 + (size_t)a1 * P1_NSUM, b1 - a1, red, tid, T1);
    reduce_columns<P2_NSUM, NTHR>(p2 + (size_t)a2 * P2_NSUM, b2 - a2, red, tid, T2);
    if (tid == 0) {
#pragma unroll
      for (int q = 0; q < P1_NSUM; ++q) ds->slice[g][q] = T1[q];
#pragma unroll
      for (int q = 0; q < P2_NSUM; ++q) ds->slice[g][P1_NSUM + q] = T2[q];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      const unsigned done = __hip_atomic_fetch_add(&ds->slices_done, 1u, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
      last = done == SOLVE_SLICES - 1;
    }
  }
  lds_sync();
  if (!last) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  if (tid < P1_NSUM + P2_NSUM) {
    double t = 0.0;
    for (int h = 0; h < SOLVE_SLICES; ++h) t += ds->slice[h][tid];
    red[tid] = t;
  }
  lds_sync();
  if (tid == 0) {
    __hip_atomic_store(&ds->slices_done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    double T1[P1_NSUM], T2[P2_NSUM];
#pragma unroll
    for (int q = 0; q < P1_NSUM; ++q) T1[q] = red[q];
#pragma unroll
    for (int q = 0; q < P2_NSUM; ++q) T2[q] = red[P1_NSUM + q];
    solve_system(T1, T2, ds, c);
  }
}

// ---------------------------------------------------------------------------
// P3: spectral combination, divide by the operator spectrum, DCT-III along y.
// ---------------------------------------------------------------------------
// UNIFORM_SYNC: every invocation passes the same workgroup barriers, also the
// ones of the k_x = 0 row-sum block below (needed where several invocations
// share a workgroup in lockstep).
template <typename TM, int NY, int NTHR, bool UNIFORM_SYNC = false>
__device__ __forceinline__ void col_solve_body(gptr<const TM> __restrict__ mid,
                                               gptr<const double> __restrict__ lamx,
                                               gptr<const double> __restrict__ lamy,
                                               gptr<const double> __restrict__ coef,
                                               gptr<TM> __restrict__ out, int nx, int chi_base,
                                               int nchi, int zeta_base, int nzeta,
                                               gptr<double> __restrict__ colsum,
                                               const OpConst c, int lin,
                                               LinesLds<TM, NY, NY>& L, int tid) {
  constexpr int LPT = NY >= NTHR ? NY / NTHR : 1;            // elements per thread
  constexpr int UPT = NY / 2 >= NTHR ? NY / 2 / NTHR : 1;    // pair units per thread
  constexpr int R = fft_radix<TM>();
  using MAP = LdsMap<TM, NY, SWZ_LINE>;
  using LS = LineSlots<NY, NTHR, R, MAP>;
  cpx<TM>* line = L.line;
  cpx<double>* rtab = L.rtab;
  const int nstrip = nx / 2;
  const int s = lin % nstrip;
  const int grp = lin / nstrip;            // 0: chi (Allen-Cahn), 1: zeta (Cahn-Hilliard)
  const size_t SS = strip_stride(NY, sizeof(TM));
  const size_t FSM = strip_field(nx, NY, sizeof(TM));
  Roots<TM, NY> rt;
  rt.init(rtab, tid, NTHR);
  const LS sl(tid);
  const int base = grp == 0 ? chi_base : zeta_base;
  const int nf = grp == 0 ? nchi : nzeta;
  const auto cf = coef + (grp == 0 ? 0 : 5);

  // Combine the x-transformed right-hand sides of this group: field by field,
  // all of a field's loads in flight together (the number of fields is a
  // compile-time constant for the step's groups: 5 for chi, 2 for zeta, and
  // 1 in a standalone solve). FP32 intermediates come in pairs: a pair whose
  // halves are consecutive slots of the group is loaded once (16 bytes a
  // row) and both halves are added in slot order, so that the sums are those
  // of the field-by-field order.
  auto combine_pairs = [&](auto inf) {
    constexpr int NF = decltype(inf)::value;
    typedef TM tm4 __attribute__((ext_vector_type(4)));
    const size_t SSP = pair_strip_stride(NY), FSP = pair_field(nx, NY);
    double ur[LPT], ui[LPT];
#pragma unroll
    for (int q = 0; q < LPT; ++q) { ur[q] = 0.0; ui[q] = 0.0; }
#pragma unroll 1
    for (int f = 0; f < NF;) {
      const int slot = base + f;
      const int p = mid_pair(slot), h = mid_half(slot);
      const bool both = h == 0 && f + 1 < NF && mid_pair(slot + 1) == p;
      const double w0 = cf[f], w1 = both ? cf[f + 1] : 0.0;
      const auto src = reinterpret_cast<gptr<const tm4>>(mid + p * FSP + (size_t)s * SSP);
      // half of the rows at a time: as many bytes in flight as one field's
      // rows, and as many registers
      constexpr int QC = LPT >= 2 ? LPT / 2 : 1;
#pragma unroll
      for (int q0 = 0; q0 < LPT; q0 += QC) {
        tm4 v[QC];
#pragma unroll
        for (int q = 0; q < QC; ++q) {
          const int jj = tid + (q0 + q) * NTHR;
          v[q] = (NY >= NTHR || jj < NY) ? src[jj] : tm4{(TM)0, (TM)0, (TM)0, (TM)0};
        }
#pragma unroll
        for (int q = 0; q < QC; ++q) {
          ur[q0 + q] += w0 * (double)(h == 0 ? v[q][0] : v[q][2]);
          ui[q0 + q] += w0 * (double)(h == 0 ? v[q][1] : v[q][3]);
          if (both) {
            ur[q0 + q] += w1 * (double)v[q][2];
            ui[q0 + q] += w1 * (double)v[q][3];
          }
        }
      }
      f += both ? 2 : 1;
    }
    static_for<LPT>([&](auto iq) {
      constexpr int q = decltype(iq)::value;
      if (NY >= NTHR || tid + q * NTHR < NY) line[sl.template mak<q>()] = {(TM)ur[q], (TM)ui[q]};
    });
  };
  auto combine_fields = [&](auto inf) {
    constexpr int NF = decltype(inf)::value;
    double ur[LPT], ui[LPT];
#pragma unroll
    for (int q = 0; q < LPT; ++q) { ur[q] = 0.0; ui[q] = 0.0; }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const double w = cf[f];
      const auto src = reinterpret_cast<gptr<const cpx<TM>>>(mid + (size_t)(base + f) * FSM +
                                                            (size_t)s * SS);
      cpx<TM> v[LPT];
#pragma unroll
      for (int q = 0; q < LPT; ++q) {
        const int jj = tid + q * NTHR;
        v[q] = (NY >= NTHR || jj < NY) ? gload<TM>(src + jj) : cpx<TM>{(TM)0, (TM)0};
      }
#pragma unroll
      for (int q = 0; q < LPT; ++q) {
        ur[q] += w * (double)v[q].re;
        ui[q] += w * (double)v[q].im;
      }
    }
    static_for<LPT>([&](auto iq) {
      constexpr int q = decltype(iq)::value;
      if (NY >= NTHR || tid + q * NTHR < NY) line[sl.template mak<q>()] = {(TM)ur[q], (TM)ui[q]};
    });
  };
  auto combine = [&](auto inf) {
    if constexpr (sizeof(TM) == 4)
      combine_pairs(inf);
    else
      combine_fields(inf);
  };
  if (nf == 5) {
    combine(std::integral_constant<int, 5>{});
  } else if (nf == 2) {
    combine(std::integral_constant<int, 2>{});
  } else {
    combine(std::integral_constant<int, 1>{});
  }
  lds_sync();
  fft_lines<TM, NY, 1, NTHR, R, MAP>(line, rt, tid);
  // FP32 lines of 8192 points and more: the divide, the inverse transform
  // and the stores form their LDS slots from a thread index of their own,
  // so that the compiler does not hold the first half's slots through them
  // (147 -> 111 registers with one butterfly per thread: two workgroups per
  // CU). Shorter lines keep the shared slots, which measured faster there.
  const int t2 = sizeof(TM) == 4 && NY >= 8192 ? opaque_vgpr(tid) : tid;
  const LS sl2(t2);
  // Per pair unit: DCT-II post-processing of both bins, divide by the operator
  // spectrum, DCT-III pre-processing of both bins (the unit holds everything
  // the inverse needs, so the line is rewritten directly).
  const double lx0 = lamx[2 * s], lx1 = lamx[2 * s + 1];
  auto op = [&](double L) {
    return grp == 0 ? c.C1 + L * (c.C2 + c.C3 * L) : c.alpha + c.lam * L;
  };
  cpx<TM> Z[UPT], Zm[UPT];
  static_for<UPT>([&](auto iq) {
    constexpr int q = decltype(iq)::value;
    const int u = t2 + q * NTHR;
    if (NY / 2 >= NTHR || u < NY / 2) {
      TM A, B, Am, Bm;
      dct2_unit<TM, NY>(line, sl2.template bin<q>(), sl2.template binm<q>(), rt, u, A, B, Am, Bm);
      const double ly = lamy[u], lym = lamy[pair_mirror<NY>(u)];
      A = (TM)((double)A * rcp64(op(lx0 + ly)));
      B = (TM)((double)B * rcp64(op(lx1 + ly)));
      Am = (TM)((double)Am * rcp64(op(lx0 + lym)));
      Bm = (TM)((double)Bm * rcp64(op(lx1 + lym)));
      // Increment form: the psi increment has zero mean (mass is conserved
      // exactly by the scheme); its (0, 0) coefficient is set, not solved.
      if (colsum && grp == 1 && s == 0 && u == 0) A = (TM)0;
      dct3_pair<TM, NY>(rt, u, A, Am, B, Bm, Z[q], Zm[q]);
    }
  });
  lds_sync();
  static_for<UPT>([&](auto iq) {
    constexpr int q = decltype(iq)::value;
    if (NY / 2 >= NTHR || t2 < NY / 2) {
      line[sl2.template nat<q>()] = Z[q];
      line[sl2.template natm<q>()] = Zm[q];
    }
  });
  lds_sync();
  fft_lines<TM, NY, 1, NTHR, R, MAP>(line, rt, t2);
  const auto dst = reinterpret_cast<gptr<cpx<TM>>>(out + (size_t)grp * FSM + (size_t)s * SS);
  TM y0[LPT];
  static_for<LPT>([&](auto iq) {
    constexpr int q = decltype(iq)::value;
    const int i = t2 + q * NTHR;
    y0[q] = (TM)0;
    if (NY >= NTHR || i < NY) {
      const cpx<TM> y = line[sl2.template out<q>()];
      gstore<TM>(dst + i, {y.re, -y.im});
      y0[q] = y.re;
    }
  });
  const bool sums_here = colsum && grp == 1 && s == 0;
  if (sums_here || (UNIFORM_SYNC && colsum)) {
    // Column k_x = 0 of the psi increment, y physical: its FP32 values sum to
    // rounding noise instead of zero. Hand the row-inverse pass FP64 targets
    // for the row sums that add up to zero, so that the increment it writes
    // has zero sum in FP64 arithmetic. (Other strips pass the barriers only.)
    double* buf = reinterpret_cast<double*>(line);   // the line is no longer read
    lds_sync();
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
      const int i = t2 + q * NTHR;
      if (sums_here && i < NY) buf[i] = (double)y0[q];
    }
    const double mean = tree_sum<NY>(buf, t2, NTHR) / NY;
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
      const int i = t2 + q * NTHR;
      if (sums_here && i < NY) colsum[i] = (double)y0[q] - mean;
    }
  }
}

// ---------------------------------------------------------------------------
// P4: DCT-III along x of the two solved fields -> phi^{n+1}, psi^{n+1}.
// ---------------------------------------------------------------------------
template <typename TM, int NX, int NTHR>
__device__ __forceinline__ void row_idct_body(gptr<const TM> __restrict__ out,
                                              gptr<double> __restrict__ phi_new,
                                              gptr<double> __restrict__ psi_new, int ny,
                                              gptr<const double> __restrict__ phi_base,
                                              gptr<const double> __restrict__ psi_base,
                                              gptr<const double> __restrict__ colsum, int j,
                                              LinesLds<TM, NX, NX>& L, int tid) {
  constexpr int CPT = NX >= NTHR ? NX / NTHR : 1;            // outputs per thread
  constexpr int UPT = NX / 2 >= NTHR ? NX / 2 / NTHR : 1;    // pair units per thread
  constexpr int R = fft_radix<TM>();
  using MAP = LdsMap<TM, NX, SWZ_LINE>;
  using LS = LineSlots<NX, NTHR, R, MAP>;
  cpx<TM>* line = L.line;
  cpx<double>* rtab = L.rtab;
  const size_t SS = strip_stride(ny, sizeof(TM));
  const size_t FSM = strip_field(NX, ny, sizeof(TM));
  Roots<TM, NX> rt;
  rt.init(rtab, tid, NTHR);
  const LS sl(tid);
  lds_sync();
  static_for<UPT>([&](auto iq) {
    constexpr int q = decltype(iq)::value;
    const int u = tid + q * NTHR;
    if (NX / 2 >= NTHR || u < NX / 2) {
      const size_t ok = mid_index(u, j, SS), om = mid_index(pair_mirror<NX>(u), j, SS);
      cpx<TM> Z, Zm;
      dct3_pair<TM, NX>(rt, u, out[ok], out[om], out[FSM + ok], out[FSM + om], Z, Zm);
      line[sl.template nat<q>()] = Z;
      line[sl.template natm<q>()] = Zm;
    }
  });
  // Increment form: level n, loaded while the transform runs when a thread
  // holds few outputs (measured: 103 -> 94 us on the 256^2 / 512^2 ensemble;
  // with 16 outputs per thread the registers cost more than the early loads
  // gain, 191 -> 196 us at N = 4096).
  constexpr bool EARLY = CPT <= 8;
  double pb[CPT], qb[CPT];
  if (EARLY && colsum) {
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const int i = tid + q * NTHR;
      const size_t o = (size_t)j * NX + (NX >= NTHR || i < NX ? i : 0);
      pb[q] = phi_base[o];
      qb[q] = psi_base[o];
    }
  }
  lds_sync();
  fft_lines<TM, NX, 1, NTHR, R, MAP>(line, rt, tid);
  if (!colsum) {
    static_for<CPT>([&](auto iq) {
      constexpr int q = decltype(iq)::value;
      const int i = tid + q * NTHR;
      if (NX >= NTHR || i < NX) {
        const cpx<TM> y = line[sl.template out<q>()];
        phi_new[(size_t)j * NX + i] = (double)y.re;
        psi_new[(size_t)j * NX + i] = -(double)y.im;
      }
    });
    return;
  }
  // Increment form: new = base + increment. The psi increment of this row is
  // shifted by a constant so that its FP64 sum equals sqrt(NX) colsum[j]
  // (orthonormal DCT-III: the row sum is sqrt(NX) times the k = 0 input).
  cpx<TM> Y[CPT];
  static_for<CPT>([&](auto iq) {
    constexpr int q = decltype(iq)::value;
    const int i = tid + q * NTHR;
    Y[q] = {(TM)0, (TM)0};
    if (NX >= NTHR || i < NX) Y[q] = line[sl.template out<q>()];
  });
  double* buf = reinterpret_cast<double*>(line);     // the line is no longer read
  lds_sync();
#pragma unroll
  for (int q = 0; q < CPT; ++q) {
    const int i = tid + q * NTHR;
    if (i < NX) buf[i] = -(double)Y[q].im;
  }
  const double shift = (sqrt((double)NX) * colsum[j] - tree_sum<NX>(buf, tid, NTHR)) / NX;
#pragma unroll
  for (int q = 0; q < CPT; ++q) {
    const int i = tid + q * NTHR;
    if (i < NX) {
      const size_t o = (size_t)j * NX + i;
      phi_new[o] = (EARLY ? pb[q] : phi_base[o]) + (double)Y[q].re;
      psi_new[o] = (EARLY ? qb[q] : psi_base[o]) + (-(double)Y[q].im + shift);
    }
  }
}

// P4 over a band of ROWS rows (row_idct_rows): each thread loads
// the band's rows of its column pairs from both strip-major fields as one
// piece per strip and field, into LDS lines in natural bin order (line r, bin
// k holding (A_k, B_k)); the DCT-III pre-processing then runs in place, unit
// by unit, since unit u reads and writes only bins u and N - u. The
// transforms, outputs and row sums are those of row_idct_body, row by row.
template <typename TM, int NX>
using RowIdctBandLds = LinesLds<TM, row_idct_rows<TM>(NX, 0) * NX, NX>;

template <typename TM, int NX>
__device__ __forceinline__ void row_idct_band_body(gptr<const TM> __restrict__ out,
                                                   gptr<double> __restrict__ phi_new,
                                                   gptr<double> __restrict__ psi_new, int ny,
                                                   gptr<const double> __restrict__ phi_base,
                                                   gptr<const double> __restrict__ psi_base,
                                                   gptr<const double> __restrict__ colsum,
                                                   int blk, RowIdctBandLds<TM, NX>& L, int tid) {
  constexpr int NTHR = row_idct_threads<TM>(NX, 0);
  constexpr int ROWS = row_idct_rows<TM>(NX, 0);
  constexpr int CPT = NX >= NTHR ? NX / NTHR : 1;            // outputs per thread and row
  constexpr int UPT = NX / 2 >= NTHR ? NX / 2 / NTHR : 1;    // strips (and units) per thread
  constexpr int R = fft_radix<TM>();
  constexpr int RS = NX * (int)sizeof(cpx<TM>) / (int)sizeof(double);   // row buffer stride
  using MAP = LdsMap<TM, NX, SWZ_ROW>;
  using LS = LineSlots<NX, NTHR, R, MAP>;
  cpx<TM>* line = L.line;
  cpx<double>* rtab = L.rtab;
  const int j0 = blk * ROWS;
  const size_t SS = strip_stride(ny, sizeof(TM));
  const size_t FSM = strip_field(NX, ny, sizeof(TM));
  Roots<TM, NX> rt;
  rt.init(rtab, tid, NTHR);
  const LS sl(tid);
  int lo[ROWS];
#pragma unroll
  for (int r = 0; r < ROWS; ++r) lo[r] = MAP::at(r * NX);
  // strip s = tid + q NTHR: rows j0 .. j0 + ROWS - 1 of bins 2 s and 2 s + 1
#pragma unroll
  for (int q = 0; q < UPT; ++q) {
    const int st = tid + q * NTHR;
    if (NX / 2 >= NTHR || st < NX / 2) {
      const size_t o = (size_t)st * SS + 2 * (size_t)j0;
      RowPiece<TM, ROWS> a, b;
      load_piece<TM, ROWS>(out + o, a);
      load_piece<TM, ROWS>(out + FSM + o, b);
      const int k0 = MAP::at(2 * st), k1 = MAP::at(2 * st + 1);
#pragma unroll
      for (int r = 0; r < ROWS; ++r) {
        line[lo[r] ^ k0] = {a.v[2 * r], b.v[2 * r]};
        line[lo[r] ^ k1] = {a.v[2 * r + 1], b.v[2 * r + 1]};
      }
    }
  }
  lds_sync();
  static_for<UPT>([&](auto iq) {
    constexpr int q = decltype(iq)::value;
    const int u = tid + q * NTHR;
    if (NX / 2 >= NTHR || u < NX / 2) {
      const int pn = sl.template nat<q>(), pm = sl.template natm<q>();
#pragma unroll
      for (int r = 0; r < ROWS; ++r) {
        const cpx<TM> x = line[lo[r] ^ pn], xm = line[lo[r] ^ pm];
        cpx<TM> Z, Zm;
        dct3_pair<TM, NX>(rt, u, x.re, xm.re, x.im, xm.im, Z, Zm);
        line[lo[r] ^ pn] = Z;
        line[lo[r] ^ pm] = Zm;
      }
    }
  });
  lds_sync();
  fft_lines<TM, NX, ROWS, NTHR, R, MAP>(line, rt, tid);
  if (!colsum) {
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      static_for<CPT>([&](auto iq) {
        constexpr int q = decltype(iq)::value;
        const int i = tid + q * NTHR;
        if (NX >= NTHR || i < NX) {
          const cpx<TM> y = line[lo[r] ^ sl.template out<q>()];
          const size_t o = (size_t)(j0 + r) * NX + i;
          phi_new[o] = (double)y.re;
          psi_new[o] = -(double)y.im;
        }
      });
    }
    return;
  }
  // Increment form: new = base + increment, the psi increment of each row
  // shifted so that its FP64 sum equals sqrt(NX) colsum[j].
  cpx<TM> Y[ROWS][CPT];
#pragma unroll
  for (int r = 0; r < ROWS; ++r) {
    static_for<CPT>([&](auto iq) {
      constexpr int q = decltype(iq)::value;
      const int i = tid + q * NTHR;
      Y[r][q] = {(TM)0, (TM)0};
      if (NX >= NTHR || i < NX) Y[r][q] = line[lo[r] ^ sl.template out<q>()];
    });
  }
  double* buf = reinterpret_cast<double*>(line);     // the lines are no longer read
  lds_sync();
#pragma unroll
  for (int r = 0; r < ROWS; ++r) {
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const int i = tid + q * NTHR;
      if (i < NX) buf[r * RS + i] = -(double)Y[r][q].im;
    }
  }
  double tot[ROWS];
  tree_sum_rows<NX, ROWS, RS>(buf, tid, NTHR, tot);
#pragma unroll
  for (int r = 0; r < ROWS; ++r) {
    const int j = j0 + r;
    const double shift = (sqrt((double)NX) * colsum[j] - tot[r]) / NX;
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const int i = tid + q * NTHR;
      if (i < NX) {
        const size_t o = (size_t)j * NX + i;
        phi_new[o] = phi_base[o] + (double)Y[r][q].re;
        psi_new[o] = psi_base[o] + (-(double)Y[r][q].im + shift);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Row DCT-II of one plain field into intermediate slot `slot` (elliptic solve).
// ---------------------------------------------------------------------------
template <typename TM, int NX>
__global__ void __launch_bounds__(line_threads(NX))
k_row_dct_field(const double* __restrict__ src, TM* __restrict__ mid, int slot, int ny,
                const int* __restrict__ skip) {
  if (skip && *skip) return;     // a converged iteration (whole workgroup)
  constexpr int NTHR = line_threads(NX);
  constexpr int CPT = NX >= NTHR ? NX / NTHR : 1;
  constexpr int UPT = NX / 2 >= NTHR ? NX / 2 / NTHR : 1;
  constexpr int R = fft_radix<TM>();
  using MAP = LdsMap<TM, NX, SWZ_LINE>;
  using LS = LineSlots<NX, NTHR, R, MAP>;
  __shared__ cpx<TM> line[NX];
  __shared__ cpx<double> rtab[Roots<TM, NX>::SIZE];
  const int tid = threadIdx.x;
  const int j = xcd_remap(blockIdx.x, gridDim.x);
  Roots<TM, NX> rt;
  rt.init(rtab, tid, NTHR);
  const LS sl(tid);
  static_for<CPT>([&](auto iq) {
    constexpr int q = decltype(iq)::value;
    const int i = tid + q * NTHR;
    if (NX >= NTHR || i < NX) line[sl.template mak<q>()] = {(TM)src[(size_t)j * NX + i], (TM)0};
  });
  lds_sync();
  fft_lines<TM, NX, 1, NTHR, R, MAP>(line, rt, tid);
  static_for<UPT>([&](auto iq) {
    constexpr int q = decltype(iq)::value;
    const int u = tid + q * NTHR;
    if (NX / 2 >= NTHR || u < NX / 2) {
      TM A, B, Am, Bm;
      dct2_unit<TM, NX>(line, sl.template bin<q>(), sl.template binm<q>(), rt, u, A, B, Am, Bm);
      mid[mid_offset<TM>(slot, u, j, NX, ny)] = A;
      mid[mid_offset<TM>(slot, pair_mirror<NX>(u), j, NX, ny)] = Am;
    }
  });
}

// ---------------------------------------------------------------------------
// Launches. Every kernel reads its arguments from a table of MemberArgs in
// device memory, so that one launch can advance several independent grids of
// the same line length (an ensemble); a single grid is a table of one. Block
// b of a launch (after the XCD renumbering) works for member idx[b / per] as
// that member's block b % per.
// ---------------------------------------------------------------------------
struct Batch {
  const MemberArgs* m;
  const int* idx;
  int per;
};

// The table, the member list and `per` are separate kernel arguments, so that
// the compiler sees the member's pointers as loaded from kernel arguments
// before any store and can treat them as global memory.
#define BATCH_PARAMS const MemberArgs* __restrict__ tab, const int* __restrict__ idx, int per

__device__ __forceinline__ const MemberArgs& batch_member(const MemberArgs* __restrict__ tab,
                                                         const int* __restrict__ idx, int per,
                                                         int& local) {
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  local = b % per;
  return tab[idx[b / per]];
}

// The stencil pass runs as a resident grid: workgroup b takes virtual blocks
// (bands) vb until all `total` are done, each XCD working through a
// contiguous range of them, so that no half-empty last wave of workgroups is
// left on the chip.
template <typename TM>
__global__ void __launch_bounds__(STENCIL_THREADS) k_stencil(BATCH_PARAMS, int total) {
  __shared__ StencilLds L;
  const int g = gridDim.x, b = blockIdx.x;
  const bool xcd = (g & 7) == 0 && (total & 7) == 0;
  const int first = xcd ? (b & 7) * (total >> 3) + (b >> 3) : b;
  const int last = xcd ? (b & 7) * (total >> 3) + (total >> 3) : total;
  const int step = xcd ? g >> 3 : g;
  for (int vb = first; vb < last; vb += step) {
    const int blk = vb % per;
    const MemberArgs& m = tab[idx[vb / per]];
    const RowArgs a{m.phn, m.phm, m.phmm, m.psn, m.psm, m.psmm};
    stencil_body<TM>(a, static_cast<gptr<TM>>(m.rm), m.part1, m.nx, m.ny, m.iters, m.k, blk,
                     m.mob_e, m.mob_n, L, threadIdx.x);
  }
}

template <typename TM, int NX, int V>
__global__ void __launch_bounds__(line_threads(NX)) k_row_dct8(BATCH_PARAMS) {
  __shared__ RowDctLds<TM, NX, V> L;
  int blk;
  const MemberArgs& m = batch_member(tab, idx, per, blk);
  row_dct8_body<TM, NX, V>(static_cast<gptr<const TM>>(m.rm), static_cast<gptr<TM>>(m.mid), m.ny,
                           blk, L, threadIdx.x);
}

template <typename TM, int NY>
__global__ void __launch_bounds__(gram_threads<TM>(NY)) k_col_gram(BATCH_PARAMS) {
  __shared__ GramLds<TM, NY> L;
  int blk;
  const MemberArgs& m = batch_member(tab, idx, per, blk);
  const OpConst o{m.k.C1, m.k.C2, m.k.C3, m.k.alpha, m.k.lam};
  col_gram_body<TM, NY>(static_cast<gptr<const TM>>(m.mid), m.lamx, m.lamy, m.part2, m.nx, o, blk,
                        L, threadIdx.x, static_cast<gptr<TM>>(m.rm));
}

template <int NTHR>
__global__ void __launch_bounds__(NTHR) k_solve(BATCH_PARAMS) {
  __shared__ SolveLds<NTHR> L;
  int blk;
  const MemberArgs& m = batch_member(tab, idx, per, blk);
  solve_body<NTHR>(m.part1, m.p1_blocks, m.part2, m.p2_rows, m.ds, m.k, L, threadIdx.x);
}

// per = SOLVE_SLICES workgroups per member
template <int NTHR>
__global__ void __launch_bounds__(NTHR) k_solve_sliced(BATCH_PARAMS) {
  __shared__ SolveLds<NTHR> L;
  int g;
  const MemberArgs& m = batch_member(tab, idx, per, g);
  solve_sliced_body<NTHR>(m.part1, m.p1_blocks, m.part2, m.p2_rows, m.ds, m.k, g, L,
                          threadIdx.x);
}

template <typename TM, int NY, int V>
__global__ void __launch_bounds__(line_threads_v<TM>(NY, V)) k_col_solve(BATCH_PARAMS) {
  __shared__ LinesLds<TM, NY, NY> L;
  int blk;
  const MemberArgs& m = batch_member(tab, idx, per, blk);
  if (m.skip && *m.skip) return;     // a converged iteration (whole workgroup)
  const OpConst o{m.k.C1, m.k.C2, m.k.C3, m.k.alpha, m.k.lam};
  col_solve_body<TM, NY, line_threads_v<TM>(NY, V)>(static_cast<gptr<const TM>>(m.mid), m.lamx, m.lamy, m.coef,
                         static_cast<gptr<TM>>(m.outc), m.nx, m.chi_base, m.nchi, m.zeta_base,
                         m.nzeta, m.colsum, o, blk, L, threadIdx.x);
}

// Row inverse variants: 0 takes a band of row_idct_rows rows per workgroup,
// 1 one row with one FFT butterfly per thread.
template <typename TM, int NX, int V>
__global__ void __launch_bounds__(row_idct_threads<TM>(NX, V),
                                  V == 0 && row_idct_threads<TM>(NX, V) == 512 ? 4 : 1)
k_row_idct(BATCH_PARAMS) {
  int blk;
  const MemberArgs& m = batch_member(tab, idx, per, blk);
  if (m.skip && *m.skip) return;     // a converged iteration (whole workgroup)
  if constexpr (V == 0) {
    __shared__ RowIdctBandLds<TM, NX> L;
    row_idct_band_body<TM, NX>(static_cast<gptr<const TM>>(m.outc), m.phi_new, m.psi_new, m.ny,
                               m.phi_base, m.psi_base, m.colsum, blk, L, threadIdx.x);
  } else {
    __shared__ LinesLds<TM, NX, NX> L;
    row_idct_body<TM, NX, line_threads_v<TM>(NX, V)>(static_cast<gptr<const TM>>(m.outc),
                                                     m.phi_new, m.psi_new, m.ny, m.phi_base,
                                                     m.psi_base, m.colsum, blk, L, threadIdx.x);
  }
}

}  // namespace ccm
