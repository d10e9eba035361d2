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

}  // namespace ccm
