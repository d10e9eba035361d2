// Initial SAVs (eq. msav_ic), modified discrete energy (eq. modified_discrete_energy)
// and mass (App. D) as row-partial reductions finished by one workgroup.
#pragma once
#include "step_kernels.hpp"

namespace ccm {

constexpr int DIAG_THREADS = 256;

enum InitSum { I_V = 0, I_SURF, I_W, I_OSM, I_NSUM };

struct DiagConst {
  double h, inv_h, inv_h2, h2, eps, beta, M0;
  double gamma_in, gamma_out, psi_in, psi_out, beta_in, beta_out;
  double gamma_surf, gamma_bend, gamma_area, theta, theta_t, lam, half_dt;
  double A;          // NaN: use the discrete surface energy of phi0
  int with_d;        // add ||d^n||^2 of the last step to the accumulator
  int periodic;      // wrap-around ghosts (periodic boundaries), else Neumann
};

// Neighbour indices of cell i on a line of n cells: the ghost copy of the
// boundary cell (Neumann), or the cell on the other side (periodic).
__device__ __forceinline__ int next_cell(int i, int n, int periodic) {
  return i + 1 < n ? i + 1 : (periodic ? 0 : n - 1);
}
__device__ __forceinline__ int prev_cell(int i, int n, int periodic) {
  return i > 0 ? i - 1 : (periodic ? n - 1 : 0);
}

// Sums of the SAV functionals of Sec. 2.2 at (phi, psi), one row per block.
__global__ void __launch_bounds__(DIAG_THREADS)
k_init_sums(const double* __restrict__ phi, const double* __restrict__ psi, double* __restrict__ part,
            int nx, int ny, DiagConst c) {
  __shared__ double red[I_NSUM * (DIAG_THREADS / 64 + 1)];
  const int tid = threadIdx.x, j = blockIdx.x;
  const int jn = next_cell(j, ny, c.periodic), js = prev_cell(j, ny, c.periodic);
  const double k32 = 0.75 * 1.4142135623730950488;
  double v[I_NSUM] = {0.0, 0.0, 0.0, 0.0};
  for (int i = tid; i < nx; i += DIAG_THREADS) {
    const int ie = next_cell(i, nx, c.periodic), iw = prev_cell(i, nx, c.periodic);
    const double p = phi[(size_t)j * nx + i];
    const double gxe = (phi[(size_t)j * nx + ie] - p) * c.inv_h;
    const double gxw = (p - phi[(size_t)j * nx + iw]) * c.inv_h;
    const double gyn = (phi[(size_t)jn * nx + i] - p) * c.inv_h;
    const double gys = (p - phi[(size_t)js * nx + i]) * c.inv_h;
    const double grad2 = 0.5 * (gxe * gxe + gxw * gxw + gyn * gyn + gys * gys);
    const double t = p * p - 1.0;
    const double vq = t - c.beta;
    v[I_V] += vq * vq / (4.0 * c.eps);
    v[I_SURF] += k32 * (0.25 * t * t / c.eps + 0.5 * c.eps * grad2);
    const double cub = p * t;
    v[I_W] += 6.0 * p * p * grad2 + cub * cub / (c.eps * c.eps);
    const double s = psi[(size_t)j * nx + i];
    const double pp = sinpi(0.5 * p);
    const double fin = 0.5 * c.gamma_in * (s - c.psi_in) * (s - c.psi_in) + c.beta_in;
    const double fout = 0.5 * c.gamma_out * (s - c.psi_out) * (s - c.psi_out) + c.beta_out;
    v[I_OSM] += (1.0 + pp) * fin + (1.0 - pp) * fout;
  }
  block_sum<I_NSUM, DIAG_THREADS>(v, red, tid);
  if (tid < I_NSUM) part[(size_t)j * I_NSUM + tid] = red[tid];
}

// V^0, U^0, W^0, Z^0 into SAV slot 0; the arc-length target A into totals[0].
__global__ void __launch_bounds__(DIAG_THREADS)
k_init_final(const double* __restrict__ part, int ny, DevScalars* __restrict__ ds, DiagConst c) {
  __shared__ double red[I_NSUM * (DIAG_THREADS / 64 + 1)];
  double T[I_NSUM];
  reduce_rows<I_NSUM, DIAG_THREADS>(part, ny, red, threadIdx.x, T);
  if (threadIdx.x != 0) return;
  const double surf = c.h2 * T[I_SURF];
  const double A = isnan(c.A) ? surf : c.A;
  ds->sav[0][0] = sqrt(c.h2 * T[I_V]);
  ds->sav[0][1] = surf - A;
  ds->sav[0][2] = sqrt(c.h2 * T[I_W]);
  ds->sav[0][3] = sqrt(c.h2 * T[I_OSM]);
  ds->totals[0] = A;
  ds->acc = 0.0;
  ds->err = 0;
  int err = 0;
  for (int i = 0; i < 4; ++i)
    if (!isfinite(ds->sav[0][i])) err |= ERR_NONFINITE;
  if (!(c.h2 * T[I_V] > 1e-280) || !(c.h2 * T[I_W] > 1e-280) || !(c.h2 * T[I_OSM] > 1e-280))
    err |= ERR_NORM;
  ds->err = err;
}

// Physical free energy of Sec. 2.1 (eq. energy_functional, densities of eq.
// energy_densities) at (phi, psi): sums of f_surf, of (g'(phi)/eps - eps
// Delta_h phi)^2 and of f_osm, one row per block (Neumann ghosts copy the
// boundary cell; periodic ones wrap around).
enum PhysSum { Q_SURF = 0, Q_BEND, Q_OSM, Q_NSUM };

__global__ void __launch_bounds__(DIAG_THREADS)
k_phys_sums(const double* __restrict__ phi, const double* __restrict__ psi,
            double* __restrict__ part, int nx, int ny, DiagConst c) {
  __shared__ double red[Q_NSUM * (DIAG_THREADS / 64 + 1)];
  const int tid = threadIdx.x, j = blockIdx.x;
  const int jn = next_cell(j, ny, c.periodic), js = prev_cell(j, ny, c.periodic);
  const double k32 = 0.75 * 1.4142135623730950488;
  double v[Q_NSUM] = {0.0, 0.0, 0.0};
  for (int i = tid; i < nx; i += DIAG_THREADS) {
    const int ie = next_cell(i, nx, c.periodic), iw = prev_cell(i, nx, c.periodic);
    const double p = phi[(size_t)j * nx + i];
    const double gxe = (phi[(size_t)j * nx + ie] - p) * c.inv_h;
    const double gxw = (p - phi[(size_t)j * nx + iw]) * c.inv_h;
    const double gyn = (phi[(size_t)jn * nx + i] - p) * c.inv_h;
    const double gys = (p - phi[(size_t)js * nx + i]) * c.inv_h;
    const double grad2 = 0.5 * (gxe * gxe + gxw * gxw + gyn * gyn + gys * gys);
    const double lap = ((gxe - gxw) + (gyn - gys)) * c.inv_h;
    const double t = p * p - 1.0;
    v[Q_SURF] += k32 * (0.25 * t * t / c.eps + 0.5 * c.eps * grad2);
    const double om = p * t / c.eps - c.eps * lap;
    v[Q_BEND] += om * om;
    const double s = psi[(size_t)j * nx + i];
    const double pp = sinpi(0.5 * p);
    const double fin = 0.5 * c.gamma_in * (s - c.psi_in) * (s - c.psi_in) + c.beta_in;
    const double fout = 0.5 * c.gamma_out * (s - c.psi_out) * (s - c.psi_out) + c.beta_out;
    v[Q_OSM] += 0.5 * ((1.0 + pp) * fin + (1.0 - pp) * fout);
  }
  block_sum<Q_NSUM, DIAG_THREADS>(v, red, tid);
  if (tid < Q_NSUM) part[(size_t)j * Q_NSUM + tid] = red[tid];
}

// F, F^surf, F^bend, F^area, F^osm and the arc length int f_surf into
// totals[3..8] (the arc-length target A is totals[0]).
__global__ void __launch_bounds__(DIAG_THREADS)
k_phys_final(const double* __restrict__ part, int ny, DevScalars* __restrict__ ds, DiagConst c) {
  __shared__ double red[Q_NSUM * (DIAG_THREADS / 64 + 1)];
  double T[Q_NSUM];
  reduce_rows<Q_NSUM, DIAG_THREADS>(part, ny, red, threadIdx.x, T);
  if (threadIdx.x != 0) return;
  const double L = c.h2 * T[Q_SURF];
  const double surf = c.gamma_surf * L;
  const double bend = c.gamma_bend * 3.0 * 1.4142135623730950488 / (16.0 * c.eps) * c.h2 * T[Q_BEND];
  const double dA = L - ds->totals[0];
  const double area = 0.5 * c.gamma_area * dA * dA;
  const double osm = c.h2 * T[Q_OSM];
  ds->totals[3] = surf + bend + area + osm;
  ds->totals[4] = surf;
  ds->totals[5] = bend;
  ds->totals[6] = area;
  ds->totals[7] = osm;
  ds->totals[8] = L;
}

// Energy norms of levels (n, n-1), ||d^n||^2 from (n, n-1, n-2), and masses.
__global__ void __launch_bounds__(DIAG_THREADS)
k_energy_sums(const double* __restrict__ p1, const double* __restrict__ p0,
              const double* __restrict__ pm, const double* __restrict__ s1,
              const double* __restrict__ s0, const double* __restrict__ sm,
              double* __restrict__ part, int nx, int ny, DiagConst c) {
  __shared__ double red[E_NSUM * (DIAG_THREADS / 64 + 1)];
  const int tid = threadIdx.x, j = blockIdx.x;
  const int jn = next_cell(j, ny, c.periodic), js = prev_cell(j, ny, c.periodic);
  double v[E_NSUM];
#pragma unroll
  for (int q = 0; q < E_NSUM; ++q) v[q] = 0.0;
  auto at = [&](const double* f, int i, int jj) { return f[(size_t)jj * nx + i]; };
  for (int i = tid; i < nx; i += DIAG_THREADS) {
    const int ie = next_cell(i, nx, c.periodic), iw = prev_cell(i, nx, c.periodic);
    // level n and the extrapolation 2 phi^n - phi^{n-1}
    const double a = at(p1, i, j), b = 2.0 * a - at(p0, i, j);
    const double ae = at(p1, ie, j), aw = at(p1, iw, j), an = at(p1, i, jn), as = at(p1, i, js);
    const double be = 2.0 * ae - at(p0, ie, j), bw = 2.0 * aw - at(p0, iw, j);
    const double bn = 2.0 * an - at(p0, i, jn), bs = 2.0 * as - at(p0, i, js);
    const double la = (ae + aw + an + as - 4.0 * a) * c.inv_h2;
    const double lb = (be + bw + bn + bs - 4.0 * b) * c.inv_h2;
    v[E_LAP1] += la * la;
    v[E_LAP2] += lb * lb;
    v[E_P1] += a * a;
    v[E_P2] += b * b;
    const double d0 = a - at(p0, i, j);
    // east and north faces of the cell (across the wrap when periodic)
    const bool face_e = c.periodic || i < nx - 1, face_n = c.periodic || j < ny - 1;
    if (face_e) {
      const double ga = (ae - a) * c.inv_h, gb = (be - b) * c.inv_h;
      const double gd = ((ae - at(p0, ie, j)) - d0) * c.inv_h;
      v[E_G1] += ga * ga; v[E_G2] += gb * gb; v[E_GD] += gd * gd;
    }
    if (face_n) {
      const double ga = (an - a) * c.inv_h, gb = (bn - b) * c.inv_h;
      const double gd = ((an - at(p0, i, jn)) - d0) * c.inv_h;
      v[E_G1] += ga * ga; v[E_G2] += gb * gb; v[E_GD] += gd * gd;
    }
    v[E_MPSI] += at(s1, i, j);
    v[E_MPHI] += a;
    if (c.with_d) {
      const double dc = at(s1, i, j) - 2.0 * at(s0, i, j) + at(sm, i, j);
      const double fc = 2.0 * at(p0, i, j) - at(pm, i, j);
      if (face_e) {
        const double de = at(s1, ie, j) - 2.0 * at(s0, ie, j) + at(sm, ie, j);
        const double fe = 2.0 * at(p0, ie, j) - at(pm, ie, j);
        const double g = (de - dc) * c.inv_h;
        v[E_D] += g * g / mobility(0.5 * (fc + fe), c.M0);
      }
      if (face_n) {
        const double dn = at(s1, i, jn) - 2.0 * at(s0, i, jn) + at(sm, i, jn);
        const double fn = 2.0 * at(p0, i, jn) - at(pm, i, jn);
        const double g = (dn - dc) * c.inv_h;
        v[E_D] += g * g / mobility(0.5 * (fc + fn), c.M0);
      }
    }
  }
  block_sum<E_NSUM, DIAG_THREADS>(v, red, tid);
  if (tid < E_NSUM) part[(size_t)j * E_NSUM + tid] = red[tid];
}

// E^{n,n-1}_mod and its parts into ds->energy; masses into ds->totals.
// energy[0] = E, energy[1..9] = bend, surf, stab, lin, V, U, W, Z, -acc.
__global__ void __launch_bounds__(DIAG_THREADS)
k_energy_final(const double* __restrict__ part, int ny, DevScalars* __restrict__ ds, int slot_n,
               int slot_m, DiagConst c) {
  __shared__ double red[E_NSUM * (DIAG_THREADS / 64 + 1)];
  double T[E_NSUM];
  reduce_rows<E_NSUM, DIAG_THREADS>(part, ny, red, threadIdx.x, T);
  if (threadIdx.x != 0) return;
  const double r2 = 1.4142135623730950488;
  const double h2 = c.h2;
  const double* S1 = ds->sav[slot_n];
  const double* S0 = ds->sav[slot_m];
  double parts[9];
  parts[0] = 0.5 * c.gamma_bend * 3.0 * r2 * c.eps / 8.0 * h2 * (T[E_LAP1] + T[E_LAP2]);
  parts[1] = 0.5 * (c.gamma_surf * 3.0 * r2 * c.eps / 4.0 + c.theta) * h2 * (T[E_G1] + T[E_G2]);
  parts[2] = -0.5 * c.theta_t * h2 * (T[E_G1] + T[E_G2] - 2.0 * T[E_GD]);
  parts[3] = 0.5 * c.gamma_surf * 3.0 * r2 * c.beta / (4.0 * c.eps) * h2 * (T[E_P1] + T[E_P2]);
  const double w[4] = {0.5 * c.gamma_surf * 1.5 * r2, 0.5 * c.gamma_area,
                       0.5 * c.gamma_bend * 3.0 * r2 / (8.0 * c.eps), 0.5};
  for (int i = 0; i < 4; ++i) {
    const double e = 2.0 * S1[i] - S0[i];
    parts[4 + i] = w[i] * (S1[i] * S1[i] + e * e);
  }
  double acc = ds->acc;
  if (c.with_d) acc += c.half_dt * c.lam * c.lam * h2 * T[E_D];
  parts[8] = -acc;
  double E = 0.0;
  for (int i = 0; i < 9; ++i) E += parts[i];
  ds->energy[0] = E;
  for (int i = 0; i < 9; ++i) ds->energy[1 + i] = parts[i];
  ds->totals[1] = h2 * T[E_MPSI];
  ds->totals[2] = h2 * T[E_MPHI];
  if (!isfinite(E)) ds->err |= ERR_NONFINITE;
}

}  // namespace ccm
