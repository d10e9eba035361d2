// Pointwise kernels around the standalone fast direct solver of App. C: the
// initial-condition relaxation of App. F (the explicit right-hand side of the
// constant-mobility Cahn-Hilliard step, the final clipping to [-1, 1]) and
// the sign alternation that turns the DCT solver into the DST one for
// homogeneous Dirichlet boundaries.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace ccm {

constexpr int SMOOTH_THREADS = 256;

// rhs = phi / dt + (M / eps) Delta_h (phi^3 - phi), five-point Laplacian
// with Neumann ghosts (the ghost copies the boundary cell, App. D). Grid:
// (ceil(nx / SMOOTH_THREADS), ny).
__global__ void __launch_bounds__(SMOOTH_THREADS)
k_smooth_rhs(const double* __restrict__ phi, double* __restrict__ rhs, int nx, int ny,
             double inv_dt, double m_over_eps, double inv_h2) {
  const int i = blockIdx.x * SMOOTH_THREADS + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= nx || j >= ny) return;
  auto g = [&](int ii, int jj) {
    ii = ii < 0 ? 0 : (ii >= nx ? nx - 1 : ii);
    jj = jj < 0 ? 0 : (jj >= ny ? ny - 1 : jj);
    const double v = phi[(size_t)jj * nx + ii];
    return v * v * v - v;
  };
  const double c = g(i, j);
  const double lap = ((g(i + 1, j) - c) - (c - g(i - 1, j)) + (g(i, j + 1) - c) -
                      (c - g(i, j - 1))) * inv_h2;
  rhs[(size_t)j * nx + i] = phi[(size_t)j * nx + i] * inv_dt + m_over_eps * lap;
}

// u <- max(-1, min(1, u)) over n values.
__global__ void __launch_bounds__(SMOOTH_THREADS) k_clip_unit(double* __restrict__ u, size_t n) {
  for (size_t k = (size_t)blockIdx.x * SMOOTH_THREADS + threadIdx.x; k < n;
       k += (size_t)gridDim.x * SMOOTH_THREADS)
    u[k] = fmin(1.0, fmax(-1.0, u[k]));
}

// out = (-1)^(i + j) in, row-major nx x ny (may alias). With it a DST-II is a
// DCT-II read in reverse order: sum_i x_i sin(pi (N - k)(2 i + 1) / (2 N)) =
// sum_i (-1)^i x_i cos(pi k (2 i + 1) / (2 N)), so the DCT kernels solve the
// homogeneous Dirichlet problem once the eigenvalues are re-indexed.
// Grid: (ceil(nx / SMOOTH_THREADS), ny).
__global__ void __launch_bounds__(SMOOTH_THREADS)
k_alternate_sign(const double* in, double* out, int nx, int ny) {
  const int i = blockIdx.x * SMOOTH_THREADS + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= nx || j >= ny) return;
  const size_t o = (size_t)j * nx + i;
  const double v = in[o];
  out[o] = ((i + j) & 1) ? -v : v;
}

}  // namespace ccm
