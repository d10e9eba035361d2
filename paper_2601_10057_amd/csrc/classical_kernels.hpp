// The classical MSAV scheme's Cahn-Hilliard solves (App. B remarks; the
// comparison system of Sec. 4), FP64: zeta x = b with the variable-coefficient
// zeta = alpha - lambda div(M_psi(phi*) grad) for the two right-hand sides of
// a step, g (explicit part) and L~ = div(M grad P~), by the conjugate gradient
// iteration preconditioned with alpha - lambda M_bar Delta_h (M_bar the mean of
// M_psi(phi*) over the cells), whose inverse is App. C's DCT solve.
//
// Both systems iterate in lock step in one set of launches; every scalar of
// the iteration lives in device memory, so the host enqueues a fixed number
// of iterations and the kernels of an iteration return at once when both
// systems have converged (a flag every block reads first, uniform over the
// block). Reductions are per-block partials summed by one workgroup in a
// fixed order, so runs repeat bit for bit.
//
// Fields are row-major FP64 N x N; system s in {0: g, 1: L~} at field s * N^2.
#pragma once
#include "step_kernels.hpp"

namespace ccm {

constexpr int CL_THREADS = 256;
constexpr int CL_BLOCKS = 1024;     // grid of the pointwise kernels (grid-stride)
constexpr int CL_NSUM = 8;          // partial sums per block row

// Scalars of the two iterations.
struct PcgScalars {
  double alpha, lam, tol;          // zeta = alpha - lam div(M grad); stop at |r| <= tol |b|
  double bnorm2[2], bsum[2];       // |b|^2 and sum b per system
  double rz[2];                    // (r, z) of the current iterate
  double a[2], beta[2];            // step length and direction update
  double rnorm2[2];
  double shift[2];                 // mean correction added to x after the iteration
  double pl[2];                    // (P~, x_s) with the mean correction
  int iters[2];
  int done[2];
  int done_all;                    // read by the solve kernels (MemberArgs::skip)
  int first;                       // the next direction is z (no beta)
};

enum ClPhase { CL_INIT = 0, CL_RZ = 1, CL_PQ = 2, CL_RR = 3, CL_FINAL = 4 };

// Sum of the blocks' partial rows: every thread gets the CL_NSUM totals.
__device__ __forceinline__ void cl_reduce(const double* __restrict__ part, int rows, double* red,
                                          double (&tot)[CL_NSUM]) {
  reduce_columns<CL_NSUM, 512>(part, rows, red, threadIdx.x, tot);
}

// x = 0, r = b (both systems), partial |b|^2 and sum b.
__global__ void __launch_bounds__(CL_THREADS)
k_cl_start(const double* __restrict__ b, double* __restrict__ x, double* __restrict__ r,
           double* __restrict__ part, size_t n, PcgScalars* __restrict__ sc) {
  __shared__ double red[CL_NSUM * (CL_THREADS / 64 + 1)];
  double v[CL_NSUM] = {};
  for (size_t o = (size_t)blockIdx.x * CL_THREADS + threadIdx.x; o < n;
       o += (size_t)gridDim.x * CL_THREADS) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const double bv = b[s * n + o];
      x[s * n + o] = 0.0;
      r[s * n + o] = bv;
      v[s] += bv * bv;
      v[2 + s] += bv;
    }
  }
  block_sum<CL_NSUM, CL_THREADS>(v, red, threadIdx.x);
  if (threadIdx.x < CL_NSUM) part[(size_t)blockIdx.x * CL_NSUM + threadIdx.x] = red[threadIdx.x];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->done[0] = sc->done[1] = 0;
    sc->done_all = 0;
    sc->iters[0] = sc->iters[1] = 0;
    sc->first = 1;
  }
}

// Partial (r, z) of both systems.
__global__ void __launch_bounds__(CL_THREADS)
k_cl_dot_rz(const double* __restrict__ r, const double* __restrict__ z, double* __restrict__ part,
            size_t n, const PcgScalars* __restrict__ sc) {
  __shared__ double red[CL_NSUM * (CL_THREADS / 64 + 1)];
  if (sc->done_all) return;
  double v[CL_NSUM] = {};
  for (size_t o = (size_t)blockIdx.x * CL_THREADS + threadIdx.x; o < n;
       o += (size_t)gridDim.x * CL_THREADS) {
    v[0] += r[o] * z[o];
    v[1] += r[n + o] * z[n + o];
  }
  block_sum<CL_NSUM, CL_THREADS>(v, red, threadIdx.x);
  if (threadIdx.x < CL_NSUM) part[(size_t)blockIdx.x * CL_NSUM + threadIdx.x] = red[threadIdx.x];
}

// The next direction p_new = z + beta p_old (p_new = z at the first
// iteration) and q = zeta p_new, with partial (p_new, q). zeta applies the
// five-point flux form with the face mobilities me (east face of each cell)
// and mn (north face); the wall faces carry no flux (Neumann).
__global__ void __launch_bounds__(CL_THREADS)
k_cl_matvec(const double* __restrict__ z, const double* __restrict__ p_old,
            double* __restrict__ p_new, double* __restrict__ q, const double* __restrict__ me,
            const double* __restrict__ mn, int nx, int ny, double inv_h2,
            double* __restrict__ part, const PcgScalars* __restrict__ sc) {
  __shared__ double red[CL_NSUM * (CL_THREADS / 64 + 1)];
  if (sc->done_all) return;
  const size_t n = (size_t)nx * ny;
  const bool first = sc->first != 0;
  const double be[2] = {first ? 0.0 : sc->beta[0], first ? 0.0 : sc->beta[1]};
  const double alpha = sc->alpha, lam = sc->lam;
  double v[CL_NSUM] = {};
  for (size_t o = (size_t)blockIdx.x * CL_THREADS + threadIdx.x; o < n;
       o += (size_t)gridDim.x * CL_THREADS) {
    const int j = (int)(o / nx), i = (int)(o - (size_t)j * nx);
    const size_t ow = i > 0 ? o - 1 : o, oe = i + 1 < nx ? o + 1 : o;
    const size_t os = j > 0 ? o - nx : o, on = j + 1 < ny ? o + nx : o;
    const double Me = i + 1 < nx ? me[o] : 0.0, Mw = i > 0 ? me[o - 1] : 0.0;
    const double Mn = j + 1 < ny ? mn[o] : 0.0, Ms = j > 0 ? mn[o - nx] : 0.0;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const size_t b0 = s * n;
      auto pn = [&](size_t k) { return z[b0 + k] + be[s] * p_old[b0 + k]; };
      const double pc = pn(o);
      const double flux = Me * (pn(oe) - pc) - Mw * (pc - pn(ow)) + Mn * (pn(on) - pc) -
                          Ms * (pc - pn(os));
      const double qv = alpha * pc - lam * flux * inv_h2;
      p_new[b0 + o] = pc;
      q[b0 + o] = qv;
      v[s] += pc * qv;
    }
  }
  block_sum<CL_NSUM, CL_THREADS>(v, red, threadIdx.x);
  if (threadIdx.x < CL_NSUM) part[(size_t)blockIdx.x * CL_NSUM + threadIdx.x] = red[threadIdx.x];
}

// x += a p, r -= a q for the systems still iterating; partial |r|^2.
__global__ void __launch_bounds__(CL_THREADS)
k_cl_update(double* __restrict__ x, double* __restrict__ r, const double* __restrict__ p,
            const double* __restrict__ q, double* __restrict__ part, size_t n,
            const PcgScalars* __restrict__ sc) {
  __shared__ double red[CL_NSUM * (CL_THREADS / 64 + 1)];
  if (sc->done_all) return;
  const double a[2] = {sc->done[0] ? 0.0 : sc->a[0], sc->done[1] ? 0.0 : sc->a[1]};
  double v[CL_NSUM] = {};
  for (size_t o = (size_t)blockIdx.x * CL_THREADS + threadIdx.x; o < n;
       o += (size_t)gridDim.x * CL_THREADS) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const size_t k = s * n + o;
      x[k] += a[s] * p[k];
      const double rv = r[k] - a[s] * q[k];
      r[k] = rv;
      v[s] += rv * rv;
    }
  }
  block_sum<CL_NSUM, CL_THREADS>(v, red, threadIdx.x);
  if (threadIdx.x < CL_NSUM) part[(size_t)blockIdx.x * CL_NSUM + threadIdx.x] = red[threadIdx.x];
}

// Partial (P~, x_s), sum x_s and sum P~ for the mean correction.
__global__ void __launch_bounds__(CL_THREADS)
k_cl_gram(const double* __restrict__ P, const double* __restrict__ x, double* __restrict__ part,
          size_t n) {
  __shared__ double red[CL_NSUM * (CL_THREADS / 64 + 1)];
  double v[CL_NSUM] = {};
  for (size_t o = (size_t)blockIdx.x * CL_THREADS + threadIdx.x; o < n;
       o += (size_t)gridDim.x * CL_THREADS) {
    const double pv = P[o], xg = x[o], xl = x[n + o];
    v[0] += pv * xg;
    v[1] += pv * xl;
    v[2] += xg;
    v[3] += xl;
    v[4] += pv;
  }
  block_sum<CL_NSUM, CL_THREADS>(v, red, threadIdx.x);
  if (threadIdx.x < CL_NSUM) part[(size_t)blockIdx.x * CL_NSUM + threadIdx.x] = red[threadIdx.x];
}

// The iteration's scalars from the partials of the kernel before (one
// workgroup of 512 threads): INIT |b|^2, sum b; RZ (r, z) and beta; PQ the
// step length a = (r, z) / (p, q); RR |r|^2 and the stopping test (an error
// bit if the last allowed iteration ends unconverged); FINAL the mean
// correction and (P~, x_s) for the 5x5 system.
template <int PHASE>
__global__ void __launch_bounds__(512)
k_cl_scalars(const double* __restrict__ part, int rows, PcgScalars* __restrict__ sc,
             DevScalars* __restrict__ ds, double cells, int last) {
  __shared__ double red[512 + CL_NSUM];
  if (PHASE != CL_INIT && PHASE != CL_FINAL && sc->done_all) return;
  double t[CL_NSUM];
  cl_reduce(part, rows, red, t);
  if (threadIdx.x != 0) return;
  if constexpr (PHASE == CL_INIT) {
    for (int s = 0; s < 2; ++s) {
      sc->bnorm2[s] = t[s];
      sc->bsum[s] = t[2 + s];
      // a zero right-hand side is solved by x = 0
      sc->done[s] = t[s] > 0.0 ? 0 : 1;
    }
    sc->done_all = sc->done[0] && sc->done[1];
  } else if constexpr (PHASE == CL_RZ) {
    for (int s = 0; s < 2; ++s) {
      if (sc->done[s]) {
        sc->beta[s] = 0.0;
        continue;
      }
      sc->beta[s] = sc->first ? 0.0 : t[s] / sc->rz[s];
      sc->rz[s] = t[s];
    }
  } else if constexpr (PHASE == CL_PQ) {
    for (int s = 0; s < 2; ++s) sc->a[s] = sc->done[s] ? 0.0 : sc->rz[s] / t[s];
    sc->first = 0;
  } else if constexpr (PHASE == CL_RR) {
    for (int s = 0; s < 2; ++s) {
      if (sc->done[s]) continue;
      sc->rnorm2[s] = t[s];
      sc->iters[s] += 1;
      if (t[s] <= sc->tol * sc->tol * sc->bnorm2[s]) sc->done[s] = 1;
    }
    sc->done_all = sc->done[0] && sc->done[1];
    if (last && !sc->done_all) ds->err |= ERR_PCG;
  } else {
    // x_s + shift_s has the exact mean sum(b_s) / (alpha N^2): summing zeta x
    // = b over the cells gives alpha sum x = sum b (the fluxes cancel).
    for (int s = 0; s < 2; ++s) {
      sc->shift[s] = (sc->bsum[s] / sc->alpha - t[2 + s]) / cells;
      sc->pl[s] = t[s] + sc->shift[s] * t[4];
      ds->cl[s] = sc->pl[s];
    }
  }
}

// psi^{n+1} = (x_g + shift_g) + c (x_L + shift_L), c = the combination
// coefficient of L~ from the 5x5 solve (App. B Step 4 recovery).
__global__ void __launch_bounds__(CL_THREADS)
k_cl_combine(const double* __restrict__ x, const PcgScalars* __restrict__ sc,
             const double* __restrict__ coef, double* __restrict__ psi_new, size_t n) {
  const double c = coef[6];
  const double sg = sc->shift[0], sl = sc->shift[1];
  for (size_t o = (size_t)blockIdx.x * CL_THREADS + threadIdx.x; o < n;
       o += (size_t)gridDim.x * CL_THREADS)
    psi_new[o] = (x[o] + sg) + c * (x[n + o] + sl);
}

// The preconditioner's constants for this step, alpha - lambda M_bar Delta_h
// (M_bar = h^2 sum M_psi(phi*) / |Omega| from the stencil partials), into the
// solve table entry (chi group: C1 = alpha, C2 = lambda M_bar, C3 = 0; zeta
// group: alpha, lambda M_bar) and the iteration's scalars.
__global__ void __launch_bounds__(512)
k_cl_setup(const double* __restrict__ p1, int rows, MemberArgs* __restrict__ pre,
           PcgScalars* __restrict__ sc, double alpha, double lam, double tol, double cells) {
  constexpr int NV = (int)P1_NSUM;
  __shared__ double red[512 + NV];
  double t[NV];
  reduce_columns<NV, 512>(p1, rows, red, threadIdx.x, t);
  if (threadIdx.x != 0) return;
  const double m_bar = t[P1_MBAR] / cells;
  pre->k.C1 = alpha;
  pre->k.C2 = lam * m_bar;
  pre->k.C3 = 0.0;
  pre->k.alpha = alpha;
  pre->k.lam = lam * m_bar;
  sc->alpha = alpha;
  sc->lam = lam;
  sc->tol = tol;
}

}  // namespace ccm
