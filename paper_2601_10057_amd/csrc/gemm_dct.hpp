// Pointwise kernels of the DCT-as-GEMM variant of the step.
//
// In this variant the four transform passes of a step run on the matrix
// cores in bfloat16 with FP32 accumulation: every FP32 operand is split into
// three bf16 parts and a product takes the six products of parts that carry
// FP32 accuracy (gemm_mfma.hpp). A direction of fewer than 2048 points is a
// dense product with the orthonormal DCT-II matrix D (D_kn = s_k cos(pi k
// (2n + 1) / 2N), s_0 = sqrt(1/N), s_k = sqrt(2/N)); a longer one takes the
// factored form of gemm_fourstep.hpp. The products only ever see the
// increment-form residuals of the mixed path. The kernels here do the
// spectral work between them: inner products, combination and divide, and
// the FP64 update of the state.
#pragma once
#include <stdint.h>

#include "step_kernels.hpp"

namespace ccm {

// FP32 -> bfloat16, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
  return __uint_as_float((uint32_t)h << 16);
}

constexpr int GEMM_THREADS = 256;

// The Parseval inner products of App. B Step 4 from the 2D spectra of the
// eight fields (field-major, [field][ky][kx], kx fastest): one row of P2Sum
// partials per workgroup, each thread taking `per_thread` consecutive cells.
__global__ void __launch_bounds__(GEMM_THREADS)
k_gemm_gram(const float* __restrict__ spec, const double* __restrict__ lamx,
            const double* __restrict__ lamy, double* __restrict__ part, int nx, int ny,
            int per_thread, StepConst c) {
  __shared__ double red[P2_NSUM * (GEMM_THREADS / 64 + 1)];
  const size_t FS = (size_t)nx * ny;
  double v[P2_NSUM];
#pragma unroll
  for (int q = 0; q < P2_NSUM; ++q) v[q] = 0.0;
  const size_t first = ((size_t)blockIdx.x * GEMM_THREADS) * per_thread + threadIdx.x;
  for (int r = 0; r < per_thread; ++r) {
    const size_t o = first + (size_t)r * GEMM_THREADS;
    if (o >= FS) break;
    const int kx = (int)(o % nx), ky = (int)(o / nx);
    const double L = lamx[kx] + lamy[ky];
    const double is = 1.0 / (c.C1 + L * (c.C2 + c.C3 * L));
    const double it = 1.0 / (c.alpha + c.lam * L);
    const double F = spec[M_F * FS + o], S = spec[M_S * FS + o], H = spec[M_H * FS + o];
    const double Q = spec[M_Q * FS + o], K = spec[M_K * FS + o], G = spec[M_G * FS + o];
    const double Lp = spec[M_L * FS + o], P = spec[M_P * FS + o];
    v[P2_FS] += F * S * is;
    v[P2_FH] += F * H * is;
    v[P2_FQ] += F * Q * is;
    v[P2_FK] += F * K * is;
    v[P2_SS] += S * S * is;
    v[P2_SH] += S * H * is;
    v[P2_SQ] += S * Q * is;
    v[P2_SK] += S * K * is;
    v[P2_HH] += H * H * is;
    v[P2_HQ] += H * Q * is;
    v[P2_HK] += H * K * is;
    v[P2_QQ] += Q * Q * is;
    v[P2_QK] += Q * K * is;
    v[P2_KK] += K * K * is;
    v[P2_PG] += P * G * it;
    v[P2_PL] += P * Lp * it;
  }
  block_sum<P2_NSUM, GEMM_THREADS>(v, red, threadIdx.x);
  if (threadIdx.x < P2_NSUM) part[(size_t)blockIdx.x * P2_NSUM + threadIdx.x] = red[threadIdx.x];
}

// Spectral combination and divide (App. B, Step 4 recovery): out[0] is the
// spectrum of the phi increment, out[1] that of the psi increment, whose
// (0, 0) coefficient is zero (its mean is carried in FP64).
__global__ void __launch_bounds__(GEMM_THREADS)
k_gemm_combine(const float* __restrict__ spec, const double* __restrict__ coef,
               const double* __restrict__ lamx, const double* __restrict__ lamy,
               float* __restrict__ out, int nx, int ny, StepConst c) {
  const size_t FS = (size_t)nx * ny;
  const size_t stride = (size_t)gridDim.x * GEMM_THREADS;
  for (size_t o = (size_t)blockIdx.x * GEMM_THREADS + threadIdx.x; o < FS; o += stride) {
    const int kx = (int)(o % nx), ky = (int)(o / nx);
    const double L = lamx[kx] + lamy[ky];
    double a = 0.0;
#pragma unroll
    for (int f = 0; f < 5; ++f) a += coef[f] * (double)spec[(M_F + f) * FS + o];
    const double b = coef[5] * (double)spec[M_G * FS + o] + coef[6] * (double)spec[M_L * FS + o];
    out[o] = (float)(a / (c.C1 + L * (c.C2 + c.C3 * L)));
    out[FS + o] = (o == 0) ? 0.0f : (float)(b / (c.alpha + c.lam * L));
  }
}

// Column k_x = 0 of the psi increment after the inverse transform along y:
// FP64 row-sum targets that add up to zero (single workgroup).
__global__ void __launch_bounds__(GEMM_THREADS)
k_gemm_colsum(const float* __restrict__ z_psi, double* __restrict__ colsum, int nx, int ny) {
  __shared__ double red[1 * (GEMM_THREADS / 64 + 1)];
  double v[1] = {0.0};
  for (int j = threadIdx.x; j < ny; j += GEMM_THREADS) v[0] += (double)z_psi[(size_t)j * nx];
  block_sum<1, GEMM_THREADS>(v, red, threadIdx.x);
  const double mean = red[0] / ny;
  for (int j = threadIdx.x; j < ny; j += GEMM_THREADS)
    colsum[j] = (double)z_psi[(size_t)j * nx] - mean;
}

// New state = level n + increments, one row per workgroup; the psi increment
// of the row is shifted so that its FP64 sum is sqrt(nx) colsum[j].
__global__ void __launch_bounds__(GEMM_THREADS)
k_gemm_finalize(const float* __restrict__ inc, const double* __restrict__ phi_base,
                const double* __restrict__ psi_base, const double* __restrict__ colsum,
                double* __restrict__ phi_new, double* __restrict__ psi_new, int nx, int ny) {
  __shared__ double red[1 * (GEMM_THREADS / 64 + 1)];
  const int j = blockIdx.x;
  const size_t FS = (size_t)nx * ny;
  const size_t row = (size_t)j * nx;
  double v[1] = {0.0};
  for (int i = threadIdx.x; i < nx; i += GEMM_THREADS) v[0] += (double)inc[FS + row + i];
  block_sum<1, GEMM_THREADS>(v, red, threadIdx.x);
  const double shift = (sqrt((double)nx) * colsum[j] - red[0]) / nx;
  for (int i = threadIdx.x; i < nx; i += GEMM_THREADS) {
    phi_new[row + i] = phi_base[row + i] + (double)inc[row + i];
    psi_new[row + i] = psi_base[row + i] + ((double)inc[FS + row + i] + shift);
  }
}

}  // namespace ccm
