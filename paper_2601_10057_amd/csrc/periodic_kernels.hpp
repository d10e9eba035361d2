// Fast direct solver for periodic boundaries (the FFT that App. C names for
// them), FP64: chi^{-1} rhs and zeta^{-1} rhs with the operators diagonal in
// the Fourier basis, eigenvalues of -Delta_h (4/h^2)(sin^2(pi kx/nx) +
// sin^2(pi ky/ny)).
//   k_per_rows     two real rows per workgroup as one complex FFT line; their
//                  half spectra (kx = 0 .. nx/2) split by conjugate symmetry
//                  into column-major complex columns;
//   k_per_cols     per column kx: FFT along y, divide by sigma and by tau,
//                  inverse FFT (conjugate, forward FFT, conjugate, 1/ny);
//   k_per_rows_inv two rows per workgroup: the full row spectrum of row j +
//                  i row j+1 from the half spectra by Hermitian symmetry,
//                  inverse FFT (1/nx), real and imaginary parts.
// Column buffers hold column kx at kx cs, cs >= ny complex values.
#pragma once
#include "step_kernels.hpp"

namespace ccm {

template <int N> __device__ __forceinline__ int per_slot(int k) {
  return LdsMap<double, N, SWZ_LINE>::at(digit_rev<N, 8>(k));
}

template <int NX>
__global__ void __launch_bounds__(line_threads(NX))
k_per_rows(const double* __restrict__ rhs, cpx<double>* __restrict__ col, int ny, size_t cs) {
  constexpr int NTHR = line_threads(NX);
  using MAP = LdsMap<double, NX, SWZ_LINE>;
  __shared__ cpx<double> line[NX];
  __shared__ cpx<double> rtab[Roots<double, NX>::SIZE];
  const int tid = threadIdx.x;
  const int j = 2 * blockIdx.x;
  if (j + 1 >= ny) return;                       // whole workgroup: no barrier skipped
  Roots<double, NX> rt;
  rt.init(rtab, tid, NTHR);
  for (int i = tid; i < NX; i += NTHR)
    line[MAP::at(i)] = {rhs[(size_t)j * NX + i], rhs[(size_t)(j + 1) * NX + i]};
  lds_sync();
  fft_lines<double, NX, 1, NTHR, 8, MAP>(line, rt, tid);
  for (int u = tid; u < NX / 2; u += NTHR) {
    const cpx<double> z = line[per_slot<NX>(u)];
    if (u == 0) {
      const cpx<double> zh = line[per_slot<NX>(NX / 2)];
      col[j] = {z.re, 0.0};
      col[j + 1] = {z.im, 0.0};
      col[(size_t)(NX / 2) * cs + j] = {zh.re, 0.0};
      col[(size_t)(NX / 2) * cs + j + 1] = {zh.im, 0.0};
    } else {
      const cpx<double> zm = line[per_slot<NX>(NX - u)];
      col[(size_t)u * cs + j] = {0.5 * (z.re + zm.re), 0.5 * (z.im - zm.im)};
      col[(size_t)u * cs + j + 1] = {0.5 * (z.im + zm.im), -0.5 * (z.re - zm.re)};
    }
  }
}

struct PerConst {
  double C1, C2, C3, alpha, lam, h;
};

template <int NY>
__global__ void __launch_bounds__(line_threads(NY))
k_per_cols(const cpx<double>* __restrict__ col, cpx<double>* __restrict__ out_chi,
           cpx<double>* __restrict__ out_zeta, int nx, size_t cs, PerConst c) {
  constexpr int NTHR = line_threads(NY);
  using MAP = LdsMap<double, NY, SWZ_LINE>;
  __shared__ cpx<double> a[NY];
  __shared__ cpx<double> b[NY];
  __shared__ cpx<double> rtab[Roots<double, NY>::SIZE];
  const int tid = threadIdx.x;
  const int kx = blockIdx.x;
  if (kx > nx / 2) return;                       // whole workgroup
  Roots<double, NY> rt;
  rt.init(rtab, tid, NTHR);
  const size_t base = (size_t)kx * cs;
  for (int i = tid; i < NY; i += NTHR) a[MAP::at(i)] = col[base + i];
  lds_sync();
  fft_lines<double, NY, 1, NTHR, 8, MAP>(a, rt, tid);
  const double sx = sinpi((double)kx / nx);
  const double lx = 4.0 / (c.h * c.h) * sx * sx;
  for (int op = 0; op < 2; ++op) {
    cpx<double>* out = op == 0 ? out_chi : out_zeta;
    if (!out) continue;                          // uniform over the workgroup
    for (int k = tid; k < NY; k += NTHR) {
      const double sy = sinpi((double)k / NY);
      const double L = lx + 4.0 / (c.h * c.h) * sy * sy;
      const double s = op == 0 ? c.C1 + L * (c.C2 + c.C3 * L) : c.alpha + c.lam * L;
      const cpx<double> x = a[per_slot<NY>(k)];
      b[MAP::at(k)] = {x.re / s, -x.im / s};     // conjugate of X / s
    }
    lds_sync();
    fft_lines<double, NY, 1, NTHR, 8, MAP>(b, rt, tid);
    for (int m = tid; m < NY; m += NTHR) {
      const cpx<double> y = b[per_slot<NY>(m)];
      out[base + m] = {y.re / NY, -y.im / NY};
    }
    lds_sync();
  }
}

template <int NX>
__global__ void __launch_bounds__(line_threads(NX))
k_per_rows_inv(const cpx<double>* __restrict__ col, double* __restrict__ out, int ny, size_t cs) {
  constexpr int NTHR = line_threads(NX);
  using MAP = LdsMap<double, NX, SWZ_LINE>;
  __shared__ cpx<double> line[NX];
  __shared__ cpx<double> rtab[Roots<double, NX>::SIZE];
  const int tid = threadIdx.x;
  const int j = 2 * blockIdx.x;
  if (j + 1 >= ny) return;                       // whole workgroup
  Roots<double, NX> rt;
  rt.init(rtab, tid, NTHR);
  for (int k = tid; k <= NX / 2; k += NTHR) {
    const cpx<double> p = col[(size_t)k * cs + j], q = col[(size_t)k * cs + j + 1];
    // Z[k] = p + i q; stored conjugated for the inverse transform
    line[MAP::at(k)] = {p.re - q.im, -(p.im + q.re)};
    if (k > 0 && k < NX / 2)                     // Z[N-k] = conj(p) + i conj(q)
      line[MAP::at(NX - k)] = {p.re + q.im, -(q.re - p.im)};
  }
  lds_sync();
  fft_lines<double, NX, 1, NTHR, 8, MAP>(line, rt, tid);
  for (int m = tid; m < NX; m += NTHR) {
    const cpx<double> z = line[per_slot<NX>(m)];
    out[(size_t)j * NX + m] = z.re / NX;
    out[(size_t)(j + 1) * NX + m] = -z.im / NX;
  }
}

// ---------------------------------------------------------------------------
// The time step with periodic boundaries (FP64). Algorithm 1 of App. B with
// the seven elliptic solves done by the solver above: chi^{-1} of f_lin (in
// place) and of S~, H, Q~, K~ (into four fields of their own), zeta^{-1} of
// g_lin and L~ (in place). The inner products of App. B Step 4 are then taken
// in physical space and the solution combined from the solved fields.
// ---------------------------------------------------------------------------
constexpr int PER_THREADS = 256;

// P2Sum partials of one grid row: (F_i, chi^{-1} F_j) for F in {S~, H, Q~, K~},
// (F_i, chi^{-1} f_lin), (P~, zeta^{-1} g_lin), (P~, zeta^{-1} L~).
// rm: the eight stencil fields (slots of Mid) with f_lin, g_lin and L~
// already replaced by their solves; xs: chi^{-1} of S~, H, Q~, K~.
__global__ void __launch_bounds__(PER_THREADS)
k_per_gram(const double* __restrict__ rm, const double* __restrict__ xs, double* __restrict__ part,
           int nx, int ny) {
  __shared__ double red[P2_NSUM * (PER_THREADS / 64 + 1)];
  const int j = blockIdx.x, tid = threadIdx.x;
  const size_t FS = (size_t)nx * ny;
  double v[P2_NSUM];
#pragma unroll
  for (int q = 0; q < P2_NSUM; ++q) v[q] = 0.0;
  for (int i = tid; i < nx; i += PER_THREADS) {
    const size_t o = (size_t)j * nx + i;
    const double f = rm[M_F * FS + o];
    const double F[4] = {rm[M_S * FS + o], rm[M_H * FS + o], rm[M_Q * FS + o], rm[M_K * FS + o]};
    const double X[4] = {xs[o], xs[FS + o], xs[2 * FS + o], xs[3 * FS + o]};
    v[P2_FS] += F[0] * f;
    v[P2_FH] += F[1] * f;
    v[P2_FQ] += F[2] * f;
    v[P2_FK] += F[3] * f;
    v[P2_SS] += F[0] * X[0];
    v[P2_SH] += F[0] * X[1];
    v[P2_SQ] += F[0] * X[2];
    v[P2_SK] += F[0] * X[3];
    v[P2_HH] += F[1] * X[1];
    v[P2_HQ] += F[1] * X[2];
    v[P2_HK] += F[1] * X[3];
    v[P2_QQ] += F[2] * X[2];
    v[P2_QK] += F[2] * X[3];
    v[P2_KK] += F[3] * X[3];
    const double P = rm[M_P * FS + o];
    v[P2_PG] += P * rm[M_G * FS + o];
    v[P2_PL] += P * rm[M_L * FS + o];
  }
  block_sum<P2_NSUM, PER_THREADS>(v, red, tid);
  if (tid < P2_NSUM) part[(size_t)j * P2_NSUM + tid] = red[tid];
}

// phi^{n+1} = sum of coef[f] times the solved chi fields (f_lin, S~, H, Q~,
// K~), psi^{n+1} = coef[5] zeta^{-1} g_lin + coef[6] zeta^{-1} L~, with the
// combination coefficients of the 5x5 solve (App. B Step 4 recovery).
__global__ void __launch_bounds__(PER_THREADS)
k_per_combine(const double* __restrict__ rm, const double* __restrict__ xs,
              const double* __restrict__ coef, double* __restrict__ phi_new,
              double* __restrict__ psi_new, size_t n) {
  const double c0 = coef[0], c1 = coef[1], c2 = coef[2], c3 = coef[3], c4 = coef[4];
  const double c5 = coef[5], c6 = coef[6];
  const size_t stride = (size_t)gridDim.x * PER_THREADS;
  for (size_t o = (size_t)blockIdx.x * PER_THREADS + threadIdx.x; o < n; o += stride) {
    phi_new[o] = c0 * rm[M_F * n + o] + c1 * xs[o] + c2 * xs[n + o] + c3 * xs[2 * n + o] +
                 c4 * xs[3 * n + o];
    psi_new[o] = c5 * rm[M_G * n + o] + c6 * rm[M_L * n + o];
  }
}

}  // namespace ccm
