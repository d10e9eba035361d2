// Host runtime of the CC-MSAV step library: parameter checks, workspace
// layout, the per-step launch sequence and the C ABI of include/ccmsav.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "ccmsav.h"
#include "diag_kernels.hpp"
#include "step_kernels.hpp"

using namespace ccm;

namespace {

constexpr int kMinLog = 4;    // 16
constexpr int kMaxLog = 13;   // 8192
constexpr int kNumSizes = kMaxLog - kMinLog + 1;
constexpr size_t kAlign = 256;
constexpr int kNumPhases = 6;   // stencil, row DCT, column Gram, 5x5 solve, column solve, row IDCT

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int log2_exact(int n) {
  if (n <= 0 || (n & (n - 1)) != 0) return -1;
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

// ---- launch tables over the line length --------------------------------------

template <typename TM> struct Launch {
  using P1 = void (*)(hipStream_t, int, const TM*, TM*, int);
  using P2 = void (*)(hipStream_t, int, const TM*, const double*, const double*, double*, int,
                      const StepConst&);
  using P3 = void (*)(hipStream_t, int, const TM*, const double*, const double*, const double*,
                      TM*, int, int, int, int, int, double*, const StepConst&);
  using P4 = void (*)(hipStream_t, int, const TM*, double*, double*, int, const double*,
                      const double*, const double*);
  using RD = void (*)(hipStream_t, int, const double*, TM*, int, int);

  template <int N>
  static void p1(hipStream_t st, int grid, const TM* rm, TM* mid, int ny) {
    hipLaunchKernelGGL((k_row_dct8<TM, N>), dim3(grid), dim3(line_threads(N)), 0, st, rm, mid, ny);
  }
  template <int N>
  static void p2(hipStream_t st, int grid, const TM* mid, const double* lx, const double* ly,
                 double* part, int nx, const StepConst& k) {
    hipLaunchKernelGGL((k_col_gram<TM, N>), dim3(grid), dim3(gram_threads(N)), 0, st, mid, lx, ly,
                       part, nx, k);
  }
  template <int N>
  static void p3(hipStream_t st, int grid, const TM* mid, const double* lx, const double* ly,
                 const double* coef, TM* out, int nx, int cb, int nc, int zb, int nz,
                 double* colsum, const StepConst& k) {
    hipLaunchKernelGGL((k_col_solve<TM, N>), dim3(grid, 2), dim3(line_threads(N)), 0, st, mid,
                       lx, ly, coef, out, nx, cb, nc, zb, nz, colsum, k);
  }
  template <int N>
  static void p4(hipStream_t st, int grid, const TM* out, double* phi, double* psi, int ny,
                 const double* phi_base, const double* psi_base, const double* colsum) {
    hipLaunchKernelGGL((k_row_idct<TM, N>), dim3(grid), dim3(line_threads(N)), 0, st, out, phi,
                       psi, ny, phi_base, psi_base, colsum);
  }
  template <int N>
  static void rd(hipStream_t st, int grid, const double* src, TM* mid, int slot, int ny) {
    hipLaunchKernelGGL((k_row_dct_field<TM, N>), dim3(grid), dim3(line_threads(N)), 0, st, src,
                       mid, slot, ny);
  }

  template <int... L> struct Tables {
    static constexpr P1 t1[] = {&p1<(1 << L)>...};
    static constexpr P2 t2[] = {&p2<(1 << L)>...};
    static constexpr P3 t3[] = {&p3<(1 << L)>...};
    static constexpr P4 t4[] = {&p4<(1 << L)>...};
    static constexpr RD trd[] = {&rd<(1 << L)>...};
  };
  using T = Tables<4, 5, 6, 7, 8, 9, 10, 11, 12, 13>;
};

}  // namespace

struct ccmsav_ctx {
  ccmsav_params p;
  int lx, ly;              // log2 nx, log2 ny
  hipStream_t stream;
  bool owns_ws;
  void* ws;
  size_t ws_bytes;
  double* phi[3];          // ring of levels, slot = level % 3
  double* psi[3];
  void* rm;                // 8 stencil fields (row-major)
  void* mid;               // 8 intermediate fields (strip-major)
  void* outc;              // 2 solved fields, x-transformed (strip-major)
  double* part1;           // ny * P1_NSUM
  double* part2;           // nx/2 * P2_NSUM
  double* parte;           // ny * max(E_NSUM, I_NSUM)
  double* lamx;            // (4/h^2) sin^2(pi k / (2 nx))
  double* lamy;
  double* colsum;          // increment form: FP64 row-sum targets of the psi increment
  double* unit_coef;       // {1, 0, 0, 0, 0, 1, 0, 0} for the standalone solve
  DevScalars* ds;
  int64_t level;
  double A;
  int last_err;
};

namespace {

size_t mid_elem(const ccmsav_params* p) { return p->precision == CCMSAV_MIXED ? 4 : 8; }

struct Layout {
  size_t state, rm, mid, outc, part1, part2, parte, lamx, lamy, colsum, unit, ds, total;
};

Layout layout(const ccmsav_params* p) {
  Layout L{};
  const size_t cells = (size_t)p->nx * p->ny;
  size_t off = 0;
  L.state = off; off = align_up(off + 6 * cells * sizeof(double));
  L.rm = off;    off = align_up(off + M_NFIELD * cells * mid_elem(p));
  L.mid = off;   off = align_up(off + M_NFIELD * cells * mid_elem(p));
  L.outc = off;  off = align_up(off + 2 * cells * mid_elem(p));
  L.part1 = off; off = align_up(off + (size_t)stencil_shape(p->nx, p->ny).blocks * P1_NSUM * sizeof(double));
  L.part2 = off; off = align_up(off + (size_t)(p->nx / 2) * P2_NSUM * sizeof(double));
  L.parte = off; off = align_up(off + (size_t)p->ny * E_NSUM * sizeof(double));
  L.lamx = off;  off = align_up(off + (size_t)p->nx * sizeof(double));
  L.lamy = off;  off = align_up(off + (size_t)p->ny * sizeof(double));
  L.colsum = off; off = align_up(off + (size_t)p->ny * sizeof(double));
  L.unit = off;  off = align_up(off + 8 * sizeof(double));
  L.ds = off;    off = align_up(off + sizeof(DevScalars));
  L.total = off;
  return L;
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }
bool finite_nonneg(double x) { return std::isfinite(x) && x >= 0.0; }

int check_params(const ccmsav_params* p) {
  if (!p) return CCMSAV_EINVAL;
  if (p->flags != 0) return CCMSAV_EINVAL;
  if (p->precision != CCMSAV_FP64 && p->precision != CCMSAV_MIXED) return CCMSAV_EUNSUPPORTED;
  if (p->nx <= 0 || p->ny <= 0) return CCMSAV_EINVAL;
  const int lx = log2_exact(p->nx), ly = log2_exact(p->ny);
  if (lx < kMinLog || lx > kMaxLog || ly < kMinLog || ly > kMaxLog) return CCMSAV_EUNSUPPORTED;
  if (!finite_pos(p->h) || !finite_pos(p->dt) || !finite_pos(p->eps) || !finite_pos(p->M_phi))
    return CCMSAV_EINVAL;
  if (!std::isfinite(p->M0) || p->M0 < 0.0 || p->M0 >= 1.0) return CCMSAV_EINVAL;
  if (!finite_nonneg(p->gamma_surf) || !finite_nonneg(p->gamma_bend) ||
      !finite_nonneg(p->gamma_area) || !finite_nonneg(p->gamma_in) ||
      !finite_nonneg(p->gamma_out) || !finite_nonneg(p->theta) || !finite_nonneg(p->lam))
    return CCMSAV_EINVAL;
  if (!std::isfinite(p->psi_in) || !std::isfinite(p->psi_out) || !std::isfinite(p->beta_in) ||
      !std::isfinite(p->beta_out) || !std::isfinite(p->beta))
    return CCMSAV_EINVAL;
  if (!std::isnan(p->A) && !std::isfinite(p->A)) return CCMSAV_EINVAL;
  return CCMSAV_OK;
}

#define HIP_TRY(expr)                                   \
  do {                                                  \
    if ((expr) != hipSuccess) return CCMSAV_EHIP;       \
  } while (0)

StepConst make_const(const ccmsav_ctx* c, bool bdf2) {
  const ccmsav_params& p = c->p;
  const double r2 = std::sqrt(2.0);
  StepConst k{};
  k.h = p.h;
  k.inv_h = 1.0 / p.h;
  k.inv_h2 = 1.0 / (p.h * p.h);
  k.h2 = p.h * p.h;
  k.eps = p.eps;
  k.beta = p.beta;
  k.M_phi = p.M_phi;
  k.M0 = p.M0;
  k.gamma_in = p.gamma_in;
  k.gamma_out = p.gamma_out;
  k.psi_in = p.psi_in;
  k.psi_out = p.psi_out;
  k.beta_in = p.beta_in;
  k.beta_out = p.beta_out;
  k.lam = p.lam;
  k.theta_t = p.theta + p.gamma_bend * 3.0 * r2 / (4.0 * p.eps);
  if (bdf2) {
    k.x0 = 2.0; k.x1 = -1.0;
    k.a0 = 2.0 / p.dt; k.a1 = -0.5 / p.dt;
    k.e0 = -4.0 / 3.0; k.e1 = 1.0 / 3.0;
    k.c0 = 4.0 / 3.0; k.c1 = -1.0 / 3.0;
    k.alpha = 1.5 / p.dt;
  } else {
    k.x0 = 1.0; k.x1 = 0.0;
    k.a0 = 1.0 / p.dt; k.a1 = 0.0;
    k.e0 = -1.0; k.e1 = 0.0;
    k.c0 = 1.0; k.c1 = 0.0;
    k.alpha = 1.0 / p.dt;
  }
  k.C1 = k.alpha + p.M_phi * p.gamma_surf * 3.0 * r2 * p.beta / (4.0 * p.eps);
  k.C2 = p.M_phi * (p.gamma_surf * 3.0 * r2 * p.eps / 4.0 + p.theta);
  k.C3 = p.M_phi * p.gamma_bend * 3.0 * r2 * p.eps / 8.0;
  k.cgs = p.M_phi * p.gamma_surf * 3.0 * r2 / 2.0;
  k.cga = p.M_phi * p.gamma_area;
  k.cgb = p.M_phi * p.gamma_bend * 3.0 * r2 / (8.0 * p.eps);
  k.cgo = p.M_phi;
  k.C1b = k.C1 - k.alpha;
  k.half_dt = 0.5 * p.dt;
  return k;
}

DiagConst make_diag(const ccmsav_ctx* c) {
  const ccmsav_params& p = c->p;
  DiagConst d{};
  d.h = p.h;
  d.inv_h = 1.0 / p.h;
  d.inv_h2 = 1.0 / (p.h * p.h);
  d.h2 = p.h * p.h;
  d.eps = p.eps;
  d.beta = p.beta;
  d.M0 = p.M0;
  d.gamma_in = p.gamma_in;
  d.gamma_out = p.gamma_out;
  d.psi_in = p.psi_in;
  d.psi_out = p.psi_out;
  d.beta_in = p.beta_in;
  d.beta_out = p.beta_out;
  d.gamma_surf = p.gamma_surf;
  d.gamma_bend = p.gamma_bend;
  d.gamma_area = p.gamma_area;
  d.theta = p.theta;
  d.theta_t = p.theta + p.gamma_bend * 3.0 * std::sqrt(2.0) / (4.0 * p.eps);
  d.lam = p.lam;
  d.half_dt = 0.5 * p.dt;
  d.A = p.A;
  return d;
}

int status_from_err(int err) {
  if (err & ERR_NONFINITE) return CCMSAV_ENONFINITE;
  if (err & (ERR_NORM | ERR_PIVOT)) return CCMSAV_EDOMAIN;
  return CCMSAV_OK;
}

int read_err(ccmsav_ctx* c, int* err) {
  HIP_TRY(hipMemcpyAsync(err, &c->ds->err, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return CCMSAV_OK;
}

// Optional per-phase timing: events[2*ph], events[2*ph+1] bracket phase ph.
struct PhaseEvents {
  hipEvent_t* ev;   // 2 * kNumPhases events of this step, or nullptr
  void mark(int i, hipStream_t s) const {
    if (ev) (void)hipEventRecord(ev[i], s);
  }
};

template <typename TM>
void enqueue_step(ccmsav_ctx* c, PhaseEvents pe = PhaseEvents{nullptr}) {
  const int nx = c->p.nx, ny = c->p.ny;
  const bool bdf2 = c->level >= 1;
  StepConst k = make_const(c, bdf2);
  const int64_t n = c->level;
  const int sn = (int)(n % 3), sm = (int)((n + 2) % 3), snew = (int)((n + 1) % 3);
  k.slot_n = sn;
  k.slot_m = bdf2 ? sm : sn;
  k.slot_new = snew;
  k.lag_d = (n >= 2) ? 1 : 0;
  const double* phn = c->phi[sn];
  const double* psn = c->psi[sn];
  const double* phm = bdf2 ? c->phi[sm] : phn;
  const double* psm = bdf2 ? c->psi[sm] : psn;
  const double* phmm = (n >= 2) ? c->phi[snew] : phm;
  const double* psmm = (n >= 2) ? c->psi[snew] : psm;
  TM* mid = static_cast<TM*>(c->mid);
  TM* outc = static_cast<TM*>(c->outc);
  using LT = typename Launch<TM>::T;
  pe.mark(0, c->stream);
  const RowArgs ra{phn, phm, phmm, psn, psm, psmm};
  TM* rm = static_cast<TM*>(c->rm);
  const StencilShape sh = stencil_shape(nx, ny);   // one row of partial sums per workgroup
  hipLaunchKernelGGL(k_stencil<TM>, dim3(sh.blocks), dim3(STENCIL_THREADS), 0, c->stream, ra, rm,
                     c->part1, nx, ny, sh.iters, k);
  pe.mark(1, c->stream);
  pe.mark(2, c->stream);
  LT::t1[c->lx - kMinLog](c->stream, ny / p1_rows<TM>(nx), rm, mid, ny);
  pe.mark(3, c->stream);
  pe.mark(4, c->stream);
  LT::t2[c->ly - kMinLog](c->stream, nx / 2, mid, c->lamx, c->lamy, c->part2, nx, k);
  pe.mark(5, c->stream);
  pe.mark(6, c->stream);
  hipLaunchKernelGGL(k_solve, dim3(1), dim3(SOLVE_THREADS), 0, c->stream, c->part1, sh.blocks,
                     c->part2, nx / 2, c->ds, k);
  pe.mark(7, c->stream);
  pe.mark(8, c->stream);
  // The FP32-transform path solves for increments over level n (see increment_form).
  double* colsum = increment_form<TM>() ? c->colsum : nullptr;
  LT::t3[c->ly - kMinLog](c->stream, nx / 2, mid, c->lamx, c->lamy, c->ds->coef, outc, nx, M_F, 5,
                          M_G, 2, colsum, k);
  pe.mark(9, c->stream);
  pe.mark(10, c->stream);
  LT::t4[c->lx - kMinLog](c->stream, ny, outc, c->phi[snew], c->psi[snew], ny, phn, psn, colsum);
  pe.mark(11, c->stream);
  c->level += 1;
}

template <typename TM>
void enqueue_solve(ccmsav_ctx* c, const double* rhs) {
  const int nx = c->p.nx, ny = c->p.ny;
  StepConst k = make_const(c, true);
  TM* mid = static_cast<TM*>(c->mid);
  TM* outc = static_cast<TM*>(c->outc);
  using LT = typename Launch<TM>::T;
  LT::trd[c->lx - kMinLog](c->stream, ny, rhs, mid, M_F, ny);
  LT::t3[c->ly - kMinLog](c->stream, nx / 2, mid, c->lamx, c->lamy, c->unit_coef, outc, nx, M_F,
                          1, M_F, 1, nullptr, k);
}

template <typename TM>
void enqueue_final_rows(ccmsav_ctx* c, double* phi_out, double* psi_out) {
  using LT = typename Launch<TM>::T;
  LT::t4[c->lx - kMinLog](c->stream, c->p.ny, static_cast<TM*>(c->outc), phi_out, psi_out,
                          c->p.ny, nullptr, nullptr, nullptr);
}

const char* kStatusText[] = {
    "success",
    "invalid argument or parameter",
    "out of memory or workspace too small",
    "HIP runtime error",
    "domain error (vanishing SAV normaliser, singular 5x5 system or non-positive mobility)",
    "non-finite value in the state",
    "unsupported grid size or precision mode",
};

}  // namespace

extern "C" {

size_t ccmsav_workspace_bytes(const ccmsav_params* p) {
  if (check_params(p) != CCMSAV_OK) return 0;
  return layout(p).total;
}

int ccmsav_init(ccmsav_ctx** out, const ccmsav_params* p, const double* phi0, const double* psi0,
                void* workspace, size_t ws_bytes, void* hip_stream) {
  if (!out || !phi0 || !psi0) return CCMSAV_EINVAL;
  *out = nullptr;
  const int pc = check_params(p);
  if (pc != CCMSAV_OK) return pc;
  const Layout L = layout(p);
  if (workspace && ws_bytes < L.total) return CCMSAV_ENOMEM;
  if (workspace && (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0) return CCMSAV_EINVAL;
  ccmsav_ctx* c = new (std::nothrow) ccmsav_ctx();
  if (!c) return CCMSAV_ENOMEM;
  c->p = *p;
  c->lx = log2_exact(p->nx);
  c->ly = log2_exact(p->ny);
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->owns_ws = workspace == nullptr;
  if (c->owns_ws) {
    if (hipMalloc(&c->ws, L.total) != hipSuccess) {
      delete c;
      return CCMSAV_ENOMEM;
    }
    c->ws_bytes = L.total;
  } else {
    c->ws = workspace;
    c->ws_bytes = ws_bytes;
  }
  char* base = static_cast<char*>(c->ws);
  const size_t cells = (size_t)p->nx * p->ny;
  double* st = reinterpret_cast<double*>(base + L.state);
  for (int s = 0; s < 3; ++s) {
    c->phi[s] = st + (size_t)(2 * s) * cells;
    c->psi[s] = st + (size_t)(2 * s + 1) * cells;
  }
  c->rm = base + L.rm;
  c->mid = base + L.mid;
  c->outc = base + L.outc;
  c->part1 = reinterpret_cast<double*>(base + L.part1);
  c->part2 = reinterpret_cast<double*>(base + L.part2);
  c->parte = reinterpret_cast<double*>(base + L.parte);
  c->lamx = reinterpret_cast<double*>(base + L.lamx);
  c->lamy = reinterpret_cast<double*>(base + L.lamy);
  c->colsum = reinterpret_cast<double*>(base + L.colsum);
  c->unit_coef = reinterpret_cast<double*>(base + L.unit);
  c->ds = reinterpret_cast<DevScalars*>(base + L.ds);
  c->level = 0;

  auto fail = [&](int code) {
    if (c->owns_ws) (void)hipFree(c->ws);
    delete c;
    return code;
  };
  // Eigenvalues of -Delta_h per direction (App. C): (4/h^2) sin^2(pi k / (2 n)).
  double* lx = new (std::nothrow) double[p->nx];
  double* ly = new (std::nothrow) double[p->ny];
  if (!lx || !ly) {
    delete[] lx;
    delete[] ly;
    return fail(CCMSAV_ENOMEM);
  }
  for (int k = 0; k < p->nx; ++k) {
    const double s = std::sin(M_PI * k / (2.0 * p->nx));
    lx[k] = 4.0 / (p->h * p->h) * s * s;
  }
  for (int k = 0; k < p->ny; ++k) {
    const double s = std::sin(M_PI * k / (2.0 * p->ny));
    ly[k] = 4.0 / (p->h * p->h) * s * s;
  }
  const double unit[8] = {1.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0};
  bool ok = hipMemcpyAsync(c->lamx, lx, p->nx * sizeof(double), hipMemcpyHostToDevice,
                           c->stream) == hipSuccess &&
            hipMemcpyAsync(c->lamy, ly, p->ny * sizeof(double), hipMemcpyHostToDevice,
                           c->stream) == hipSuccess &&
            hipMemcpyAsync(c->unit_coef, unit, sizeof(unit), hipMemcpyHostToDevice, c->stream) ==
                hipSuccess &&
            hipMemsetAsync(c->ds, 0, sizeof(DevScalars), c->stream) == hipSuccess &&
            hipMemcpyAsync(c->phi[0], phi0, cells * sizeof(double), hipMemcpyDefault,
                           c->stream) == hipSuccess &&
            hipMemcpyAsync(c->psi[0], psi0, cells * sizeof(double), hipMemcpyDefault,
                           c->stream) == hipSuccess;
  if (ok) ok = hipStreamSynchronize(c->stream) == hipSuccess;
  delete[] lx;
  delete[] ly;
  if (!ok) return fail(CCMSAV_EHIP);

  DiagConst d = make_diag(c);
  hipLaunchKernelGGL(k_init_sums, dim3(p->ny), dim3(DIAG_THREADS), 0, c->stream, c->phi[0],
                     c->psi[0], c->parte, p->nx, p->ny, d);
  hipLaunchKernelGGL(k_init_final, dim3(1), dim3(DIAG_THREADS), 0, c->stream, c->parte, p->ny,
                     c->ds, d);
  if (hipGetLastError() != hipSuccess) return fail(CCMSAV_EHIP);
  int err = 0;
  double A = 0.0;
  if (hipMemcpyAsync(&A, &c->ds->totals[0], sizeof(double), hipMemcpyDeviceToHost, c->stream) !=
          hipSuccess ||
      read_err(c, &err) != CCMSAV_OK)
    return fail(CCMSAV_EHIP);
  c->A = A;
  c->p.A = A;
  const int st0 = status_from_err(err);
  if (st0 != CCMSAV_OK) return fail(st0);
  *out = c;
  return CCMSAV_OK;
}

int ccmsav_step(ccmsav_ctx* c, int32_t nsteps) {
  if (!c || nsteps < 0) return CCMSAV_EINVAL;
  for (int32_t s = 0; s < nsteps; ++s) {
    if (c->p.precision == CCMSAV_MIXED)
      enqueue_step<float>(c);
    else
      enqueue_step<double>(c);
  }
  if (hipGetLastError() != hipSuccess) return CCMSAV_EHIP;
  return CCMSAV_OK;
}

int ccmsav_profile_steps(ccmsav_ctx* c, int32_t nsteps, double* ms_per_phase) {
  if (!c || nsteps <= 0 || nsteps > 100000 || !ms_per_phase) return CCMSAV_EINVAL;
  const int nev = 2 * kNumPhases;
  hipEvent_t* ev = new (std::nothrow) hipEvent_t[(size_t)nev * nsteps];
  if (!ev) return CCMSAV_ENOMEM;
  int created = 0;
  int rc = CCMSAV_OK;
  for (; created < nev * nsteps; ++created) {
    if (hipEventCreate(&ev[created]) != hipSuccess) {
      rc = CCMSAV_EHIP;
      break;
    }
  }
  if (rc == CCMSAV_OK) {
    for (int32_t s = 0; s < nsteps; ++s) {
      PhaseEvents pe{ev + (size_t)nev * s};
      if (c->p.precision == CCMSAV_MIXED)
        enqueue_step<float>(c, pe);
      else
        enqueue_step<double>(c, pe);
    }
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess)
      rc = CCMSAV_EHIP;
  }
  if (rc == CCMSAV_OK) {
    for (int ph = 0; ph < kNumPhases; ++ph) {
      double tot = 0.0;
      for (int32_t s = 0; s < nsteps; ++s) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, ev[(size_t)nev * s + 2 * ph],
                                ev[(size_t)nev * s + 2 * ph + 1]) != hipSuccess)
          rc = CCMSAV_EHIP;
        tot += ms;
      }
      ms_per_phase[ph] = tot / nsteps;
    }
  }
  for (int i = 0; i < created; ++i) (void)hipEventDestroy(ev[i]);
  delete[] ev;
  if (rc != CCMSAV_OK) return rc;
  return ccmsav_sync(c);
}

int ccmsav_sync(ccmsav_ctx* c) {
  if (!c) return CCMSAV_EINVAL;
  int err = 0;
  const int r = read_err(c, &err);
  if (r != CCMSAV_OK) return r;
  return status_from_err(err);
}

static int run_diag(ccmsav_ctx* c, bool energy) {
  const int64_t n = c->level;
  const int sn = (int)(n % 3), sm = (int)((n + 2) % 3), smm = (int)((n + 1) % 3);
  DiagConst d = make_diag(c);
  d.with_d = (energy && n >= 2) ? 1 : 0;
  const double* p1 = c->phi[sn];
  const double* p0 = n >= 1 ? c->phi[sm] : p1;
  const double* pm = n >= 2 ? c->phi[smm] : p0;
  const double* s1 = c->psi[sn];
  const double* s0 = n >= 1 ? c->psi[sm] : s1;
  const double* sm_ = n >= 2 ? c->psi[smm] : s0;
  hipLaunchKernelGGL(k_energy_sums, dim3(c->p.ny), dim3(DIAG_THREADS), 0, c->stream, p1, p0, pm,
                     s1, s0, sm_, c->parte, c->p.nx, c->p.ny, d);
  hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(DIAG_THREADS), 0, c->stream, c->parte,
                     c->p.ny, c->ds, sn, n >= 1 ? sm : sn, d);
  if (hipGetLastError() != hipSuccess) return CCMSAV_EHIP;
  return CCMSAV_OK;
}

int ccmsav_energy(ccmsav_ctx* c, double* E_mod, double* parts) {
  if (!c || !E_mod) return CCMSAV_EINVAL;
  if (c->level < 1) return CCMSAV_EINVAL;
  int r = run_diag(c, true);
  if (r != CCMSAV_OK) return r;
  double e[10];
  HIP_TRY(hipMemcpyAsync(e, c->ds->energy, sizeof(e), hipMemcpyDeviceToHost, c->stream));
  int err = 0;
  r = read_err(c, &err);
  if (r != CCMSAV_OK) return r;
  *E_mod = e[0];
  if (parts)
    for (int i = 0; i < 9; ++i) parts[i] = e[1 + i];
  if (err & ERR_MOBILITY) return CCMSAV_EDOMAIN;
  return status_from_err(err);
}

int ccmsav_mass(ccmsav_ctx* c, double* mass_psi, double* mass_phi) {
  if (!c) return CCMSAV_EINVAL;
  int r = run_diag(c, false);
  if (r != CCMSAV_OK) return r;
  double t[3];
  HIP_TRY(hipMemcpyAsync(t, c->ds->totals, sizeof(t), hipMemcpyDeviceToHost, c->stream));
  int err = 0;
  r = read_err(c, &err);
  if (r != CCMSAV_OK) return r;
  if (mass_psi) *mass_psi = t[1];
  if (mass_phi) *mass_phi = t[2];
  return status_from_err(err);
}

int ccmsav_get_fields(ccmsav_ctx* c, double* phi, double* psi) {
  if (!c) return CCMSAV_EINVAL;
  const size_t bytes = (size_t)c->p.nx * c->p.ny * sizeof(double);
  const int s = (int)(c->level % 3);
  if (phi) HIP_TRY(hipMemcpyAsync(phi, c->phi[s], bytes, hipMemcpyDefault, c->stream));
  if (psi) HIP_TRY(hipMemcpyAsync(psi, c->psi[s], bytes, hipMemcpyDefault, c->stream));
  return ccmsav_sync(c);
}

int ccmsav_get_savs(ccmsav_ctx* c, double out8[8]) {
  if (!c || !out8) return CCMSAV_EINVAL;
  double sav[3][4];
  HIP_TRY(hipMemcpyAsync(sav, c->ds->sav, sizeof(sav), hipMemcpyDeviceToHost, c->stream));
  const int r = ccmsav_sync(c);
  const int64_t n = c->level;
  const int sn = (int)(n % 3), sm = n >= 1 ? (int)((n + 2) % 3) : sn;
  for (int i = 0; i < 4; ++i) {
    out8[i] = sav[sn][i];
    out8[4 + i] = sav[sm][i];
  }
  return r;
}

int64_t ccmsav_level(const ccmsav_ctx* c) { return c ? c->level : -1; }

int ccmsav_elliptic_solve(ccmsav_ctx* c, const double* rhs, double* out_chi, double* out_zeta) {
  if (!c || !rhs) return CCMSAV_EINVAL;
  if (c->p.precision == CCMSAV_MIXED)
    enqueue_solve<float>(c, rhs);
  else
    enqueue_solve<double>(c, rhs);
  // The row DCT-III writes both results; an output that is not requested goes
  // to intermediate slots 2-3, which the solve does not read.
  double* tmp = reinterpret_cast<double*>(static_cast<char*>(c->mid) +
                                          2 * (size_t)c->p.nx * c->p.ny * mid_elem(&c->p));
  double* a = out_chi ? out_chi : tmp;
  double* b = out_zeta ? out_zeta : tmp;
  if (c->p.precision == CCMSAV_MIXED)
    enqueue_final_rows<float>(c, a, b);
  else
    enqueue_final_rows<double>(c, a, b);
  if (hipGetLastError() != hipSuccess) return CCMSAV_EHIP;
  return CCMSAV_OK;
}

int ccmsav_destroy(ccmsav_ctx* c) {
  if (!c) return CCMSAV_EINVAL;
  (void)hipStreamSynchronize(c->stream);
  if (c->owns_ws) (void)hipFree(c->ws);
  delete c;
  return CCMSAV_OK;
}

const char* ccmsav_strerror(int code) {
  if (code > 0 || code < CCMSAV_EUNSUPPORTED) return "unknown status";
  return kStatusText[-code];
}

}  // extern "C"
