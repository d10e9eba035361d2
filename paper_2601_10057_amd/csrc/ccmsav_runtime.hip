// Host runtime of the CC-MSAV step library: parameter checks, workspace
// layout, the per-step launch sequence and the C ABI of include/ccmsav.h.
//
// A context advances one or more independent grids ("members") in lock step.
// Members with the same grid shape form a size class; every kernel of a step
// is one launch per size class that covers all of its members, with the
// per-member arguments read from tables in device memory (one table per kind
// of step: the BDF1 first step, the first BDF2 step, and the three phases of
// the three-level state ring). Optionally the steady-state steps are captured
// once into a HIP graph of three steps and replayed.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "ccmsav.h"
#include "classical_kernels.hpp"
#include "diag_kernels.hpp"
#include "gemm_dct.hpp"
#include "gemm_fourstep.hpp"
#include "gemm_mfma.hpp"
#include "persist_kernels.hpp"
#include "periodic_kernels.hpp"
#include "smooth_kernels.hpp"
#include "step_kernels.hpp"

using namespace ccm;

namespace {

constexpr int kMinLog = 4;    // 16
constexpr int kMaxLog = 13;   // 8192
constexpr size_t kAlign = 256;
constexpr int kNumPhases = 6;   // stencil, row DCT, column Gram, 5x5 solve, column solve, row IDCT
constexpr int kMaxMembers = 4096;
// Argument tables: 0 = level 0 (BDF1), 1 = level 1 (first BDF2 step, no
// lagged ||d||^2), 2 + r = level n >= 2 with n % 3 == r; 5 = standalone solve;
// 6 = the classical scheme's preconditioner solve.
constexpr int kNumTables = 7;
constexpr int kSolveTable = 5;
constexpr int kPcgTable = 6;
// Classical scheme: default PCG tolerance (relative residual) and iterations.
constexpr double kPcgTol = 1e-12;
constexpr int kPcgMaxIter = 40;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
constexpr size_t align_up_c(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int log2_exact(int n) {
  if (n <= 0 || (n & (n - 1)) != 0) return -1;
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

int table_of_level(int64_t n) { return n == 0 ? 0 : (n == 1 ? 1 : 2 + (int)(n % 3)); }

// A level whose step uses table t (t < kSolveTable).
int64_t level_of_table(int t) {
  if (t <= 1) return t;
  const int r = t - 2;
  return r == 0 ? 3 : (r == 1 ? 4 : 2);
}

// ---- launch tables over the line length --------------------------------------

// Autotuned kernels: row DCT (band height), column solve and row inverse
// (threads per line); kNumVariants launch variants each.
constexpr int kNumTuned = 3;
constexpr int kNumVariants = 2;
enum Tuned { TUNE_ROW_DCT = 0, TUNE_COL_SOLVE = 1, TUNE_ROW_IDCT = 2 };

template <typename TM> struct Launch {
  using K = void (*)(hipStream_t, int, const Batch&);

  template <int N, int V>
  static void row_dct(hipStream_t st, int grid, const Batch& b) {
    hipLaunchKernelGGL((k_row_dct8<TM, N, V>), dim3(grid), dim3(line_threads(N)), 0, st, b.m,
                       b.idx, b.per);
  }
  template <int N>
  static void gram(hipStream_t st, int grid, const Batch& b) {
    hipLaunchKernelGGL((k_col_gram<TM, N>), dim3(grid), dim3(gram_threads<TM>(N)), 0, st, b.m, b.idx,
                       b.per);
  }
  template <int N, int V>
  static void col_solve(hipStream_t st, int grid, const Batch& b) {
    hipLaunchKernelGGL((k_col_solve<TM, N, V>), dim3(grid), dim3(line_threads_v<TM>(N, V)), 0, st,
                       b.m, b.idx, b.per);
  }
  template <int N, int V>
  static void row_idct(hipStream_t st, int grid, const Batch& b) {
    hipLaunchKernelGGL((k_row_idct<TM, N, V>), dim3(grid), dim3(row_idct_threads<TM>(N, V)), 0, st,
                       b.m, b.idx, b.per);
  }
  using RD = void (*)(hipStream_t, int, const double*, TM*, int, int, const int*);
  template <int N>
  static void rd(hipStream_t st, int grid, const double* src, TM* mid, int slot, int ny,
                 const int* skip) {
    hipLaunchKernelGGL((k_row_dct_field<TM, N>), dim3(grid), dim3(line_threads(N)), 0, st, src,
                       mid, slot, ny, skip);
  }

  template <int... L> struct Tables {
    static constexpr K t_row_dct[kNumVariants][sizeof...(L)] = {{&row_dct<(1 << L), 0>...},
                                                                {&row_dct<(1 << L), 1>...}};
    static constexpr K t_gram[] = {&gram<(1 << L)>...};
    static constexpr K t_col_solve[kNumVariants][sizeof...(L)] = {
        {&col_solve<(1 << L), 0>...}, {&col_solve<(1 << L), 1>...}};
    static constexpr K t_row_idct[kNumVariants][sizeof...(L)] = {
        {&row_idct<(1 << L), 0>...}, {&row_idct<(1 << L), 1>...}};
    static constexpr RD t_rd[] = {&rd<(1 << L)>...};
  };
  using T = Tables<4, 5, 6, 7, 8, 9, 10, 11, 12, 13>;
};

// Rows per workgroup of the row DCT for variant v (host side of p1_rows_v).
int row_dct_rows(int precision, int nx, int v) {
  return precision == CCMSAV_FP64 ? p1_rows_v<double>(nx, v) : p1_rows_v<float>(nx, v);
}

size_t mid_elem(int precision) { return precision == CCMSAV_FP64 ? 8 : 4; }
bool is_gemm(int precision) { return precision == CCMSAV_MIXED_GEMM_BF16X3; }
// Solved in increment form (FP32 transforms of FP64-formed residuals).
bool is_inc(int precision) { return precision != CCMSAV_FP64; }
// Cells per thread of the GEMM variant's inner-product kernel.
constexpr int kGramPerThread = 16;
size_t gemm_gram_blocks(const ccmsav_params* p) {
  const size_t cells = (size_t)p->nx * p->ny;
  const size_t per_block = (size_t)GEMM_THREADS * kGramPerThread;
  return (cells + per_block - 1) / per_block;
}
bool is_periodic(const ccmsav_params* p) { return (p->flags & CCMSAV_FLAG_PERIODIC) != 0; }
bool is_classical(const ccmsav_params* p) { return (p->flags & CCMSAV_FLAG_CLASSICAL) != 0; }
bool is_persistent(const ccmsav_params* p) { return (p->flags & CCMSAV_FLAG_PERSISTENT) != 0; }
// Rows of inner-product partials: one per strip (spectral path), per block of
// cells (DCT-as-GEMM) or per grid row (periodic step, physical space).
size_t p2_rows(const ccmsav_params* p) {
  if (is_periodic(p)) return (size_t)p->ny;
  return is_gemm(p->precision) ? gemm_gram_blocks(p) : (size_t)(p->nx / 2);
}

// DCT-as-GEMM variant: a direction of n points takes the factored transform
// (gemm_fourstep.hpp) with n = N1 N2, N1 returned here, where both products
// fill the matrix-core tiles (N1 >= 32 for K, N2 >= 64 for M); 0: the dense
// product with the n x n DCT matrix.
int fs_n1(int n) { return n >= 4096 ? 64 : n == 2048 ? 32 : 0; }
// bf16 parts of the factored transform's four matrices (three parts each),
// and the offset of its two twiddle tables behind them.
size_t fs_mat_elems(int n1, int n2) {
  return 3 * (6 * (size_t)n1 * n1 + 4 * (size_t)n2 * n2);
}
size_t fs_table_offset(int n1, int n2) { return align_up(fs_mat_elems(n1, n2) * sizeof(uint16_t)); }
// Bytes of a direction's transform data: D and D^T (three bf16 parts each), or
// the factored transform's matrices and its two tables of n float2 factors.
size_t gemm_mat_bytes(int n) {
  const int n1 = fs_n1(n);
  if (n1 == 0) return 6 * (size_t)n * n * sizeof(uint16_t);
  return fs_table_offset(n1, n / n1) + 2 * (size_t)n * sizeof(float2);
}
bool uses_fs(const ccmsav_params* p) { return fs_n1(p->nx) != 0 || fs_n1(p->ny) != 0; }

struct Layout {
  size_t state, rm, mid, outc, part1, part2, parte, lamx, lamy, colsum, unit, ds;
  size_t dx, dy;   // GEMM variant: the transform matrices per direction, as bf16 parts
  size_t fs;       // GEMM variant, factored transforms: complex work buffer
  size_t psol;     // periodic step: chi^{-1} of S~, H, Q~, K~ (4 FP64 fields)
  size_t cl, clpart, clsc;   // classical scheme: PCG fields, partial sums, scalars
  size_t total;
};

Layout layout(const ccmsav_params* p) {
  Layout L{};
  const size_t cells = (size_t)p->nx * p->ny;
  const size_t me = mid_elem(p->precision);
  size_t off = 0;
  L.state = off; off = align_up(off + 6 * cells * sizeof(double));
  L.rm = off;    off = align_up(off + M_NFIELD * cells * me);
  // strip-major intermediates (padded strips; the DCT-as-GEMM variant uses
  // the first nx ny values of each field slot in its own layout)
  const size_t sf = strip_field(p->nx, p->ny, (int)me);
  L.mid = off;   off = align_up(off + M_NFIELD * sf * me);
  L.outc = off;  off = align_up(off + 2 * sf * me);
  L.part1 = off;
  off = align_up(off + (size_t)stencil_shape(p->nx, p->ny).blocks * P1_NSUM * sizeof(double));
  L.part2 = off; off = align_up(off + p2_rows(p) * P2_NSUM * sizeof(double));
  L.parte = off; off = align_up(off + (size_t)p->ny * E_NSUM * sizeof(double));
  L.lamx = off;  off = align_up(off + (size_t)p->nx * sizeof(double));
  L.lamy = off;  off = align_up(off + (size_t)p->ny * sizeof(double));
  L.colsum = off; off = align_up(off + (size_t)p->ny * sizeof(double));
  L.unit = off;  off = align_up(off + 8 * sizeof(double));
  L.ds = off;    off = align_up(off + sizeof(DevScalars));
  if (is_gemm(p->precision)) {
    L.dx = off;    off = align_up(off + gemm_mat_bytes(p->nx));
    L.dy = off;    off = align_up(off + gemm_mat_bytes(p->ny));
    // Re and Im planes of all M_NFIELD fields
    if (uses_fs(p)) { L.fs = off; off = align_up(off + 2 * M_NFIELD * cells * sizeof(float)); }
  }
  if (is_periodic(p)) {
    L.psol = off;  off = align_up(off + 4 * cells * sizeof(double));
  }
  if (is_classical(p)) {
    // x, r, p (two buffers), q, z for both systems, and the two face mobilities
    L.cl = off;     off = align_up(off + 14 * cells * sizeof(double));
    L.clpart = off; off = align_up(off + (size_t)CL_BLOCKS * CL_NSUM * sizeof(double));
    L.clsc = off;   off = align_up(off + sizeof(PcgScalars));
  }
  L.total = off;
  return L;
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }
bool finite_nonneg(double x) { return std::isfinite(x) && x >= 0.0; }

int check_params(const ccmsav_params* p) {
  if (!p) return CCMSAV_EINVAL;
  if ((p->flags & ~(CCMSAV_FLAG_GRAPH | CCMSAV_FLAG_BDF1 | CCMSAV_FLAG_PERIODIC |
                     CCMSAV_FLAG_CLASSICAL | CCMSAV_FLAG_PERSISTENT)) != 0)
    return CCMSAV_EINVAL;
  if (p->precision != CCMSAV_FP64 && p->precision != CCMSAV_MIXED &&
      p->precision != CCMSAV_MIXED_GEMM_BF16X3)
    return CCMSAV_EUNSUPPORTED;
  if (is_gemm(p->precision) && (p->flags & CCMSAV_FLAG_GRAPH)) return CCMSAV_EUNSUPPORTED;
  if (p->nx <= 0 || p->ny <= 0) return CCMSAV_EINVAL;
  const int lx = log2_exact(p->nx), ly = log2_exact(p->ny);
  if (lx < kMinLog || lx > kMaxLog || ly < kMinLog || ly > kMaxLog) return CCMSAV_EUNSUPPORTED;
  // the matrix-core products take tiles of at least 64 along each direction
  if (is_gemm(p->precision) && (p->nx < 64 || p->ny < 64)) return CCMSAV_EUNSUPPORTED;
  // the periodic step: FP64, the FFT solver's grids (up to 4096), no graph
  if (is_periodic(p) && (p->precision != CCMSAV_FP64 || lx > 12 || ly > 12 ||
                         (p->flags & CCMSAV_FLAG_GRAPH)))
    return CCMSAV_EUNSUPPORTED;
  // the classical scheme: FP64, Neumann boundaries, no graph
  if (is_classical(p) && (p->precision != CCMSAV_FP64 || is_periodic(p) ||
                          (p->flags & CCMSAV_FLAG_GRAPH)))
    return CCMSAV_EUNSUPPORTED;
  // the persistent launch: FP32 transforms, the CC-MSAV Neumann step, the
  // grid sizes its kernel is built for
  if (is_persistent(p) && (p->precision != CCMSAV_MIXED || is_periodic(p) || is_classical(p) ||
                           lx < PS_MIN_LOG || lx > PS_MAX_LOG || ly < PS_MIN_LOG ||
                           ly > PS_MAX_LOG))
    return CCMSAV_EUNSUPPORTED;
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

// All members of one context share the precision and the flags.
int check_batch(int32_t nmemb, const ccmsav_params* p) {
  if (nmemb <= 0 || nmemb > kMaxMembers || !p) return CCMSAV_EINVAL;
  for (int32_t m = 0; m < nmemb; ++m) {
    const int r = check_params(&p[m]);
    if (r != CCMSAV_OK) return r;
    if (p[m].precision != p[0].precision || p[m].flags != p[0].flags) return CCMSAV_EINVAL;
  }
  if (nmemb > 1 && (is_gemm(p[0].precision) || is_periodic(&p[0]) || is_classical(&p[0])))
    return CCMSAV_EUNSUPPORTED;
  return CCMSAV_OK;
}

// Workspace of a context: the members' regions back to back, then the
// argument tables and the member index lists.
struct BatchLayout {
  std::vector<size_t> member;   // offset of each member's region
  size_t args, idx, bar, total;
};

BatchLayout batch_layout(int32_t nmemb, const ccmsav_params* p) {
  BatchLayout B;
  size_t off = 0;
  for (int32_t m = 0; m < nmemb; ++m) {
    B.member.push_back(off);
    off = align_up(off + layout(&p[m]).total);
  }
  B.args = off;
  off = align_up(off + (size_t)kNumTables * nmemb * sizeof(MemberArgs));
  B.idx = off;
  off = align_up(off + (size_t)nmemb * sizeof(int));
  B.bar = off;                  // grid barrier of the persistent launch
  off = align_up(off + sizeof(GridBarrier));
  B.total = off;
  return B;
}

#define HIP_TRY(expr)                                   \
  do {                                                  \
    if ((expr) != hipSuccess) return CCMSAV_EHIP;       \
  } while (0)

StepConst make_const(const ccmsav_params& p, bool bdf2) {
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
  k.periodic = is_periodic(&p) ? 1 : 0;
  k.classical = is_classical(&p) ? 1 : 0;
  return k;
}

DiagConst make_diag(const ccmsav_params& p) {
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
  d.periodic = is_periodic(&p) ? 1 : 0;
  return d;
}

int status_from_err(int err) {
  if (err & ERR_NONFINITE) return CCMSAV_ENONFINITE;
  if (err & ERR_BARRIER) return CCMSAV_EBARRIER;
  if (err & ERR_PCG) return CCMSAV_ECONVERGE;
  if (err & (ERR_NORM | ERR_PIVOT)) return CCMSAV_EDOMAIN;
  return CCMSAV_OK;
}

// Optional per-phase timing: events[2*ph], events[2*ph+1] bracket phase ph.
struct PhaseEvents {
  hipEvent_t* ev;   // 2 * kNumPhases events of this step, or nullptr
  void mark(int i, hipStream_t s) const {
    if (ev) (void)hipEventRecord(ev[i], s);
  }
};

// One member (one grid) of a context.
// The matrices and twiddle tables of a factored transform along one
// direction (n = N1 N2, gemm_fourstep.hpp): bf16 parts (hi, mid, lo), row-major
// with the product dimension contiguous. Rows 2k and 2k + 1 of the
// complex-output matrices give the real and imaginary part of output k; the
// columns of complex inputs are [real parts, imaginary parts].
struct FsMats {
  int l1 = 0, l2 = 0;   // log2 of N1 and N2; l1 = 0: dense products
  MfMat d1;             // forward step 1: W_N1^(n1 k1), 2 N1 x N1
  MfMat d2;             // forward step 3: sqrt(2/N) exp(-i pi k2 (4 n2 + 1) / 2 N2), N2 x 2 N2
  MfMat d1i;            // inverse step 1: sqrt(N/2) exp(-i pi a1 (4 b1 + 1) / 2 N1), 2 N1 x 2 N1
  MfMat d2i;            // inverse step 3: W_N2^(a2 b2) / N, N2 x 2 N2
  const float2* twf;    // forward step 2: exp(-i pi k1 (4 n2 + 1) / 2N), [k1][n2]
  const float2* twi;    // inverse step 2: exp(-i pi a2 (4 b1 + 1) / 2N), [b1][a2]
};

struct Member {
  ccmsav_params p;
  int lx, ly;
  double* phi[3];          // ring of levels, slot = level % 3
  double* psi[3];
  void* rm;
  void* mid;
  void* outc;
  double* part1;
  double* part2;
  double* parte;
  double* lamx;
  double* lamy;
  double* colsum;
  double* unit_coef;       // {1, 0, 0, 0, 0, 1, 0, 0} for the standalone solve
  DevScalars* ds;
  StencilShape sh;
  // GEMM variant: per direction, the orthonormal DCT-II matrix D and its
  // transpose as bf16 parts, row-major (dense directions), or the matrices of
  // the factored transform (fsx, fsy) and its work buffer
  FsMats fsx, fsy;
  float* fs_w;
  MfMat dx, dxt, dy, dyt;
  // periodic step: chi^{-1} of S~, H, Q~, K~
  double* psol;
  // classical scheme: PCG fields (x, r, p0, p1, q, z; two systems each) and
  // the face mobilities, partial sums, scalars
  double* cl_x;
  double* cl_r;
  double* cl_p[2];
  double* cl_q;
  double* cl_z;
  double* mob_e;
  double* mob_n;
  double* cl_part;
  PcgScalars* cl_sc;
};

// Members with one grid shape; d_idx lists their indices in device memory.
struct SizeClass {
  int lx, ly;
  int count;
  const int* d_idx;
  StencilShape sh;
  int var[kNumTuned];            // chosen launch variant of each tuned kernel
  float tune_ms[kNumTuned][kNumVariants];   // best measured time of each variant
};

}  // namespace

struct ccmsav_ctx {
  std::vector<Member> mem;
  std::vector<SizeClass> cls;
  int precision = CCMSAV_FP64;
  bool graph = false;
  bool bdf1 = false;       // every step with the BDF1 scheme (CCMSAV_FLAG_BDF1)
  bool periodic = false;   // periodic boundaries (CCMSAV_FLAG_PERIODIC)
  bool classical = false;  // classical MSAV scheme (CCMSAV_FLAG_CLASSICAL)
  bool persistent = false; // one launch per step (CCMSAV_FLAG_PERSISTENT)
  unsigned spin_limit = 1u << 22;
  int ps_grid = 0;         // resident workgroups of the persistent kernel
  PersistPlan ps_plan{};
  GridBarrier* bar = nullptr;
  double pcg_tol = kPcgTol;
  int pcg_max_iter = kPcgMaxIter;
  hipStream_t stream = nullptr;
  bool owns_ws = false;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  MemberArgs* d_args = nullptr;      // kNumTables tables of mem.size() entries
  std::vector<MemberArgs> h_args;
  int64_t level = 0;
  bool tuned = false;      // launch variants chosen (at the first step)
  // graph replay of three steady-state steps
  hipStream_t gstream = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // graph branches of the size classes beyond the first
  std::vector<hipStream_t> bstream;
  std::vector<hipEvent_t> bevent;
  hipEvent_t ev_fork = nullptr;
  // resident workgroups of the stencil pass on this device ([0] FP32, [1] FP64 intermediates)
  int stencil_slots[2] = {0, 0};
};

namespace {

MemberArgs member_args(const Member& m, int precision, int table) {
  MemberArgs a{};
  const bool inc = is_inc(precision);
  a.rm = to_global(m.rm);
  a.mid = to_global(m.mid);
  a.outc = to_global(m.outc);
  a.part1 = to_global(m.part1);
  a.part2 = to_global(m.part2);
  a.lamx = to_global<const double>(m.lamx);
  a.lamy = to_global<const double>(m.lamy);
  a.ds = to_global(m.ds);
  a.nx = m.p.nx;
  a.ny = m.p.ny;
  a.mob_e = to_global(m.mob_e);
  a.mob_n = to_global(m.mob_n);
  a.iters = m.sh.iters;
  a.p1_blocks = m.sh.blocks;
  a.p2_rows = (int)p2_rows(&m.p);
  if (table == kPcgTable) {
    // The classical scheme's preconditioner alpha - lambda M_bar Delta_h for
    // the residuals of both systems: slot M_F through the chi group and slot
    // M_G through the zeta group, the constants written on the device each
    // step (k_cl_setup), outputs z of system 0 and 1; the kernels return at
    // once after both systems have converged.
    a.k = make_const(m.p, true);
    a.coef = to_global<const double>(m.unit_coef);
    a.chi_base = M_F;
    a.nchi = 1;
    a.zeta_base = M_G;
    a.nzeta = 1;
    a.phi_new = to_global(m.cl_z);
    a.psi_new = to_global(m.cl_z ? m.cl_z + (size_t)m.p.nx * m.p.ny : nullptr);
    a.skip = to_global<const int>(m.cl_sc ? &m.cl_sc->done_all : nullptr);
    return a;
  }
  if (table == kSolveTable) {
    // chi^{-1} and zeta^{-1} of the single field in slot M_F (App. C).
    a.k = make_const(m.p, true);
    a.coef = to_global<const double>(m.unit_coef);
    a.chi_base = M_F;
    a.nchi = 1;
    a.zeta_base = M_F;
    a.nzeta = 1;
    return a;
  }
  const int64_t lv = level_of_table(table);
  // BDF2 from level 1 on, or the BDF1 scheme (App. B remark) at every level.
  const bool bdf2 = lv >= 1 && (m.p.flags & CCMSAV_FLAG_BDF1) == 0;
  const int sn = (int)(lv % 3), sm = (int)((lv + 2) % 3), snew = (int)((lv + 1) % 3);
  a.k = make_const(m.p, bdf2);
  a.k.slot_n = sn;
  a.k.slot_m = bdf2 ? sm : sn;
  a.k.slot_new = snew;
  a.k.lag_d = bdf2 && lv >= 2 ? 1 : 0;
  const double* phn = m.phi[sn];
  const double* psn = m.psi[sn];
  const double* phm = bdf2 ? m.phi[sm] : phn;
  const double* psm = bdf2 ? m.psi[sm] : psn;
  a.phn = to_global(phn);
  a.psn = to_global(psn);
  a.phm = to_global(phm);
  a.psm = to_global(psm);
  a.phmm = to_global<const double>(bdf2 && lv >= 2 ? m.phi[snew] : phm);
  a.psmm = to_global<const double>(bdf2 && lv >= 2 ? m.psi[snew] : psm);
  a.phi_new = to_global(m.phi[snew]);
  a.psi_new = to_global(m.psi[snew]);
  a.coef = to_global<const double>(m.ds->coef);
  a.chi_base = M_F;
  a.nchi = 5;
  a.zeta_base = M_G;
  a.nzeta = 2;
  // The FP32-transform path solves for increments over level n (increment_form).
  a.phi_base = inc ? a.phn : nullptr;
  a.psi_base = inc ? a.psn : nullptr;
  a.colsum = inc ? to_global(m.colsum) : nullptr;
  return a;
}

// Workgroups of a stencil launch over `total` bands: as many as stay resident
// on the device at once (a multiple of 8, one share per XCD), or `total` if
// that is smaller. Measured at N = 4096, the resident grid helps the FP32
// path (313 -> 303 us) and slows the FP64 one (411 -> 422 us), which keeps
// one workgroup per band.
int stencil_grid(ccmsav_ctx* c, bool fp64, int total) {
  if (fp64) return total;
  int& slots = c->stencil_slots[fp64 ? 1 : 0];
  if (slots == 0) {
    int dev = 0, cus = 0, per_cu = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cus = 0;
    const hipError_t e =
        fp64 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_stencil<double>,
                                                             STENCIL_THREADS, 0)
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_stencil<float>,
                                                            STENCIL_THREADS, 0);
    slots = (e == hipSuccess && cus > 0 && per_cu > 0) ? (cus * per_cu) & ~7 : -1;
  }
  return (slots <= 0 || total <= slots) ? total : slots;
}

// Autotuner: at the first step every variant of each tuned kernel is run
// (they compute bit-identical results from the same inputs, so the step's
// outcome does not depend on the order) and timed with HIP events on the
// context's stream; the fastest (the least of its repetitions) is kept for
// all later steps. The repetitions alternate between the variants, so that
// clock and cache drift over the tuning launches weigh on all of them.
constexpr int kTuneReps = 5;
struct Tuner {
  bool on = false;
  std::vector<hipEvent_t> ev;   // [class][kernel][variant][rep][2]
  size_t at(size_t k, int t, int v, int r, int e) const {
    return (((k * kNumTuned + t) * kNumVariants + v) * kTuneReps + r) * 2 + e;
  }
};

template <typename TM, typename F>
void run_tuned(ccmsav_ctx* c, Tuner& tu, size_t ki, int t, hipStream_t st, F launch) {
  const SizeClass& k = c->cls[ki];
  if (!tu.on) {
    launch(k.var[t]);
    return;
  }
  for (int r = 0; r < kTuneReps; ++r)
    for (int v = 0; v < kNumVariants; ++v) {
      (void)hipEventRecord(tu.ev[tu.at(ki, t, v, r, 0)], st);
      launch(v);
      (void)hipEventRecord(tu.ev[tu.at(ki, t, v, r, 1)], st);
    }
}

// The classical scheme's two variable-coefficient solves of one step (FP64,
// one member), after the stencil pass has written g_lin (with lambda
// div(M grad psi*)), L~, P~ and the face mobilities: the preconditioner's
// constants, x = 0, r = b, z = P^{-1} r, then pcg_max_iter iterations of
// {p = z + beta p, q = zeta p; a; x += a p, r -= a q; stop test; z = P^{-1} r;
// (r, z), beta}, whose kernels return at once once both systems have met the
// tolerance, and the inner products (P~, x_s) with the mean correction. The
// intermediate fields serve as the preconditioner's scratch before the row
// DCT of the step overwrites them.
void enqueue_classical_solves(ccmsav_ctx* c, int table, hipStream_t st) {
  const Member& m = c->mem[0];
  const SizeClass& k = c->cls[0];
  const int nx = m.p.nx, ny = m.p.ny;
  const size_t n = (size_t)nx * ny;
  const MemberArgs* pre = c->d_args + (size_t)kPcgTable * c->mem.size();
  const StepConst& sc = c->h_args[(size_t)table * c->mem.size()].k;
  double* rm = static_cast<double*>(m.rm);
  const double* b = rm + (size_t)M_G * n;          // g_lin and L~ are consecutive slots
  const int rows = CL_BLOCKS;
  using LT = Launch<double>::T;
  auto precondition = [&]() {
    LT::t_rd[m.lx - kMinLog](st, ny, m.cl_r, static_cast<double*>(m.mid), M_F, ny,
                             &m.cl_sc->done_all);
    LT::t_rd[m.lx - kMinLog](st, ny, m.cl_r + n, static_cast<double*>(m.mid), M_G, ny,
                             &m.cl_sc->done_all);
    LT::t_col_solve[k.var[TUNE_COL_SOLVE]][m.ly - kMinLog](st, nx, Batch{pre, k.d_idx, nx});
    const int vi = k.var[TUNE_ROW_IDCT];
    const int per = ny / row_idct_rows<double>(nx, vi);
    LT::t_row_idct[vi][m.lx - kMinLog](st, per, Batch{pre, k.d_idx, per});
    hipLaunchKernelGGL(k_cl_dot_rz, dim3(CL_BLOCKS), dim3(CL_THREADS), 0, st, m.cl_r, m.cl_z,
                       m.cl_part, n, m.cl_sc);
    hipLaunchKernelGGL(k_cl_scalars<CL_RZ>, dim3(1), dim3(512), 0, st, m.cl_part, rows, m.cl_sc,
                       m.ds, (double)n, 0);
  };
  hipLaunchKernelGGL(k_cl_setup, dim3(1), dim3(512), 0, st, m.part1, m.sh.blocks,
                     const_cast<MemberArgs*>(pre), m.cl_sc, sc.alpha, m.p.lam, c->pcg_tol,
                     (double)n);
  hipLaunchKernelGGL(k_cl_start, dim3(CL_BLOCKS), dim3(CL_THREADS), 0, st, b, m.cl_x, m.cl_r,
                     m.cl_part, n, m.cl_sc);
  hipLaunchKernelGGL(k_cl_scalars<CL_INIT>, dim3(1), dim3(512), 0, st, m.cl_part, rows, m.cl_sc,
                     m.ds, (double)n, 0);
  precondition();
  for (int it = 0; it < c->pcg_max_iter; ++it) {
    double* p_old = m.cl_p[it & 1];
    double* p_new = m.cl_p[(it + 1) & 1];
    hipLaunchKernelGGL(k_cl_matvec, dim3(CL_BLOCKS), dim3(CL_THREADS), 0, st, m.cl_z, p_old,
                       p_new, m.cl_q, m.mob_e, m.mob_n, nx, ny, 1.0 / (m.p.h * m.p.h), m.cl_part,
                       m.cl_sc);
    hipLaunchKernelGGL(k_cl_scalars<CL_PQ>, dim3(1), dim3(512), 0, st, m.cl_part, rows, m.cl_sc,
                       m.ds, (double)n, 0);
    hipLaunchKernelGGL(k_cl_update, dim3(CL_BLOCKS), dim3(CL_THREADS), 0, st, m.cl_x, m.cl_r,
                       p_new, m.cl_q, m.cl_part, n, m.cl_sc);
    hipLaunchKernelGGL(k_cl_scalars<CL_RR>, dim3(1), dim3(512), 0, st, m.cl_part, rows, m.cl_sc,
                       m.ds, (double)n, it + 1 == c->pcg_max_iter ? 1 : 0);
    if (it + 1 < c->pcg_max_iter) precondition();
  }
  hipLaunchKernelGGL(k_cl_gram, dim3(CL_BLOCKS), dim3(CL_THREADS), 0, st,
                     rm + (size_t)M_P * n, m.cl_x, m.cl_part, n);
  hipLaunchKernelGGL(k_cl_scalars<CL_FINAL>, dim3(1), dim3(512), 0, st, m.cl_part, rows, m.cl_sc,
                     m.ds, (double)n, 0);
}

// The 5x5 kernel of `count` members of class k, with the thread count and
// the slicing of their grid size (every path of a grid uses the same, so
// results agree). Grids of 2048^2 cells and more reduce their thousands of
// partial rows over SOLVE_SLICES workgroups each: measured on one MI355X,
// 24.5 -> 15.0 us at N = 4096, 17.8 -> 14.2 us at N = 2048 and 48 -> 17 us
// at N = 8192, while at N = 1024 one workgroup is faster (11.5 against
// 12.8 us).
void launch_solve(hipStream_t st, const SizeClass& k, int count, const MemberArgs* tab) {
  const size_t cells = (size_t)1 << (k.lx + k.ly);
  if (cells >= (size_t)2048 * 2048)
    hipLaunchKernelGGL(k_solve_sliced<SOLVE_THREADS>, dim3(count * SOLVE_SLICES),
                       dim3(SOLVE_THREADS), 0, st, tab, k.d_idx, SOLVE_SLICES);
  else if (solve_threads(cells) == SOLVE_THREADS)
    hipLaunchKernelGGL(k_solve<SOLVE_THREADS>, dim3(count), dim3(SOLVE_THREADS), 0, st, tab,
                       k.d_idx, 1);
  else
    hipLaunchKernelGGL(k_solve<SOLVE_THREADS_SMALL>, dim3(count), dim3(SOLVE_THREADS_SMALL), 0,
                       st, tab, k.d_idx, 1);
}

template <typename TM>
void enqueue_step_kind(ccmsav_ctx* c, int table, hipStream_t st, PhaseEvents pe, Tuner& tu,
                       int only) {
  const MemberArgs* tab = c->d_args + (size_t)table * c->mem.size();
  using LT = typename Launch<TM>::T;
  // `only` >= 0 restricts the step to one size class (a branch of the graph).
  auto skip = [&](size_t ki) { return only >= 0 && (int)ki != only; };
  pe.mark(0, st);
  for (size_t ki = 0; ki < c->cls.size(); ++ki) {
    if (skip(ki)) continue;
    const SizeClass& k = c->cls[ki];
    const int total = k.count * k.sh.blocks;
    hipLaunchKernelGGL(k_stencil<TM>, dim3(stencil_grid(c, sizeof(TM) == 8, total)),
                       dim3(STENCIL_THREADS), 0, st, tab, k.d_idx, k.sh.blocks, total);
  }
  if constexpr (sizeof(TM) == 8) {
    if (c->classical) enqueue_classical_solves(c, table, st);
  }
  pe.mark(1, st);
  pe.mark(2, st);
  for (size_t ki = 0; ki < c->cls.size(); ++ki) {
    if (skip(ki)) continue;
    const SizeClass& k = c->cls[ki];
    run_tuned<TM>(c, tu, ki, TUNE_ROW_DCT, st, [&](int v) {
      const int per = (1 << k.ly) / row_dct_rows(c->precision, 1 << k.lx, v);
      LT::t_row_dct[v][k.lx - kMinLog](st, k.count * per, Batch{tab, k.d_idx, per});
    });
  }
  pe.mark(3, st);
  pe.mark(4, st);
  for (size_t ki = 0; ki < c->cls.size(); ++ki) {
    if (skip(ki)) continue;
    const SizeClass& k = c->cls[ki];
    const int per = (1 << k.lx) / 2;
    LT::t_gram[k.ly - kMinLog](st, k.count * per, Batch{tab, k.d_idx, per});
  }
  pe.mark(5, st);
  pe.mark(6, st);
  for (size_t ki = 0; ki < c->cls.size(); ++ki) {
    if (skip(ki)) continue;
    const SizeClass& k = c->cls[ki];
    launch_solve(st, k, k.count, tab);
  }
  pe.mark(7, st);
  pe.mark(8, st);
  for (size_t ki = 0; ki < c->cls.size(); ++ki) {
    if (skip(ki)) continue;
    const SizeClass& k = c->cls[ki];
    run_tuned<TM>(c, tu, ki, TUNE_COL_SOLVE, st, [&](int v) {
      const int per = 1 << k.lx;     // two groups (chi, zeta) per strip of two columns
      LT::t_col_solve[v][k.ly - kMinLog](st, k.count * per, Batch{tab, k.d_idx, per});
    });
  }
  pe.mark(9, st);
  pe.mark(10, st);
  for (size_t ki = 0; ki < c->cls.size(); ++ki) {
    if (skip(ki)) continue;
    const SizeClass& k = c->cls[ki];
    run_tuned<TM>(c, tu, ki, TUNE_ROW_IDCT, st, [&](int v) {
      const int per = (1 << k.ly) / row_idct_rows<TM>(1 << k.lx, v);
      LT::t_row_idct[v][k.lx - kMinLog](st, k.count * per, Batch{tab, k.d_idx, per});
    });
  }
  if (c->classical) {
    // psi^{n+1} from the iterative solves (the row inverse wrote the
    // spectral zeta group's result, which the classical scheme does not use)
    const Member& m = c->mem[0];
    const int lv = (int)level_of_table(table);
    hipLaunchKernelGGL(k_cl_combine, dim3(CL_BLOCKS), dim3(CL_THREADS), 0, st, m.cl_x, m.cl_sc,
                       m.ds->coef, m.psi[(lv + 1) % 3], (size_t)m.p.nx * m.p.ny);
  }
  pe.mark(11, st);
}

// ---- DCT-as-GEMM variant ------------------------------------------------------

// One product of the DCT-as-GEMM variant (gemm_mfma.hpp) with the largest
// tiles that divide the grid, the data operand read as XL says, stored
// through the epilogue EPI.
template <int MODE, int EPI = EPI_STORE, int XL = XL_PLAIN>
void mf_product(hipStream_t st, const MfMat& d, const float* x, float* out, int M, int N, int K,
                int ldx, int ldc, size_t sx, size_t sc, int batch,
                FsArgs fa = FsArgs{0, 0, 0, nullptr}) {
  // the factored transforms' first products along x and the inverse one
  // along y (short K) take 64-row tiles, three blocks per CU instead of two:
  // at N = 8192 the inverse column product runs 14-16% faster, the row ones
  // within a few percent; the forward column product was 5% slower with
  // them and keeps 128 rows
  constexpr bool narrow = EPI == EPI_TW_M || (EPI == EPI_TW_Z && XL == XL_Z_COLS);
  const int bm = narrow ? 64 : mf_tile(M), bn = mf_tile(N);
  const dim3 grid((unsigned)(batch * (M / bm) * (N / bn)));
  if (bm == 128 && bn == 128)
    hipLaunchKernelGGL((k_gemm_bf16x3<MODE, 128, 128, EPI, XL>), grid, dim3(MF_THREADS), 0,
                       st, d, x, out, M, N, K, ldx, ldc, sx, sc, fa);
  else if (bm == 128)
    hipLaunchKernelGGL((k_gemm_bf16x3<MODE, 128, 64, EPI, XL>), grid, dim3(MF_THREADS), 0,
                       st, d, x, out, M, N, K, ldx, ldc, sx, sc, fa);
  else if (bn == 128)
    hipLaunchKernelGGL((k_gemm_bf16x3<MODE, 64, 128, EPI, XL>), grid, dim3(MF_THREADS), 0,
                       st, d, x, out, M, N, K, ldx, ldc, sx, sc, fa);
  else
    hipLaunchKernelGGL((k_gemm_bf16x3<MODE, 64, 64, EPI, XL>), grid, dim3(MF_THREADS), 0,
                       st, d, x, out, M, N, K, ldx, ldc, sx, sc, fa);
}

// DCT-II (inverse = false) or DCT-III along x of `lines` contiguous rows,
// src -> dst: one product with D (D^T), or the factored transform.
void gemm_dct_rows(const Member& m, hipStream_t st, const float* src, float* dst, int lines,
                   bool inverse) {
  const int nx = m.p.nx;
  const FsMats& f = m.fsx;
  if (f.l1 == 0) {
    mf_product<MF_ROW>(st, inverse ? m.dxt : m.dx, src, dst, nx,
                                                 lines, nx, nx, nx, 0, 0, 1);
    return;
  }
  const int n1 = 1 << f.l1, n2 = 1 << f.l2;
  float* t = m.fs_w;                                   // T: 2 nx per line
  const FsArgs fa{f.l1, f.l2, 0, inverse ? f.twi : f.twf};
  if (!inverse) {
    mf_product<MF_COL, EPI_TW_M, XL_MAKHOUL_ROWS>(st, f.d1, src, t, n2, 2 * n1, n1, 0, n2,
                                                      0, 2 * (size_t)nx, lines, fa);
    mf_product<MF_ROW, EPI_POST_ROWS>(st, f.d2, t, dst, n2, lines * n1, 2 * n2, 2 * n2, 0,
                                          0, 0, 1, fa);
  } else {
    mf_product<MF_COL, EPI_TW_M, XL_Z_ROWS>(st, f.d1i, src, t, n2, 2 * n1, 2 * n1, 0, n2, 0,
                                                2 * (size_t)nx, lines, fa);
    mf_product<MF_ROW, EPI_IPOST_ROWS>(st, f.d2i, t, dst, n2, lines * n1, 2 * n2, 2 * n2, 0,
                                           0, 0, 1, fa);
  }
}

// DCT-II or DCT-III along y of `fields` fields of ny x nx values, src -> dst.
void gemm_dct_cols(const Member& m, hipStream_t st, const float* src, float* dst, int fields,
                   bool inverse) {
  const int nx = m.p.nx, ny = m.p.ny;
  const size_t cells = (size_t)nx * ny;
  const FsMats& f = m.fsy;
  if (f.l1 == 0) {
    mf_product<MF_COL>(st, inverse ? m.dyt : m.dy, src, dst, nx, ny,
                                                 ny, nx, nx, cells, cells, fields);
    return;
  }
  const int n1 = 1 << f.l1, n2 = 1 << f.l2, lx = m.lx;
  const int ld = n2 * nx;                  // stride of k1 in T
  const size_t sv = 2 * (size_t)n2 * nx;   // one k1 block of T
  float* t = m.fs_w;                       // T: 2 cells per field
  const FsArgs fa{f.l1, f.l2, lx, inverse ? f.twi : f.twf};
  for (int fl = 0; fl < fields; ++fl) {
    if (!inverse)
      mf_product<MF_COL, EPI_TW_Z, XL_MAKHOUL_COLS>(st, f.d1, src + fl * cells,
                                                        t + 2 * fl * cells, nx, 2 * n1, n1, 0,
                                                        ld, 0, (size_t)nx, n2, fa);
    else
      mf_product<MF_COL, EPI_TW_Z, XL_Z_COLS>(st, f.d1i, src + fl * cells,
                                                  t + 2 * fl * cells, nx, 2 * n1, 2 * n1, 0, ld,
                                                  0, (size_t)nx, n2, fa);
  }
  if (!inverse)
    mf_product<MF_COL, EPI_POST_COLS>(st, f.d2, t, dst, nx, n2, 2 * n2, nx, 0, sv, 0,
                                          fields * n1, fa);
  else
    mf_product<MF_COL, EPI_IPOST_COLS>(st, f.d2i, t, dst, nx, n2, 2 * n2, nx, 0, sv, 0,
                                           fields * n1, fa);
}

// One step of the single member with every transform on the matrix cores.
// Data flow (FP32, row-major [field][y][x]): stencil -> rm; rows: DCT along x
// rm -> mid (the 8 fields' rows stacked); columns: DCT along y mid -> rm (2D
// spectra); inner products, 5x5; combine -> outc; columns: inverse along y
// outc -> mid; rows: inverse along x mid -> outc; state update.
int enqueue_step_gemm(ccmsav_ctx* c, int64_t level, hipStream_t st, PhaseEvents pe) {
  const Member& m = c->mem[0];
  const SizeClass& k = c->cls[0];
  const int nx = m.p.nx, ny = m.p.ny;
  const size_t cells = (size_t)nx * ny;
  const MemberArgs* tab = c->d_args + (size_t)table_of_level(level) * c->mem.size();
  const MemberArgs& ha = c->h_args[(size_t)table_of_level(level) * c->mem.size()];
  float* rm = static_cast<float*>(m.rm);
  float* mid = static_cast<float*>(m.mid);
  float* outc = static_cast<float*>(m.outc);
  pe.mark(0, st);
  hipLaunchKernelGGL(k_stencil<float>, dim3(stencil_grid(c, false, k.sh.blocks)),
                     dim3(STENCIL_THREADS), 0, st, tab, k.d_idx, k.sh.blocks, k.sh.blocks);
  pe.mark(1, st);
  pe.mark(2, st);
  gemm_dct_rows(m, st, rm, mid, M_NFIELD * ny, false);
  pe.mark(3, st);
  pe.mark(4, st);
  gemm_dct_cols(m, st, mid, rm, M_NFIELD, false);
  hipLaunchKernelGGL(k_gemm_gram, dim3((unsigned)gemm_gram_blocks(&m.p)), dim3(GEMM_THREADS), 0,
                     st, rm, m.lamx, m.lamy, m.part2, nx, ny, kGramPerThread, ha.k);
  pe.mark(5, st);
  pe.mark(6, st);
  launch_solve(st, k, 1, tab);
  pe.mark(7, st);
  pe.mark(8, st);
  hipLaunchKernelGGL(k_gemm_combine, dim3((unsigned)std::min<size_t>(cells / GEMM_THREADS + 1, 8192)),
                     dim3(GEMM_THREADS), 0, st, rm, m.ds->coef, m.lamx, m.lamy, outc, nx, ny,
                     ha.k);
  gemm_dct_cols(m, st, outc, mid, 2, true);
  hipLaunchKernelGGL(k_gemm_colsum, dim3(1), dim3(GEMM_THREADS), 0, st, mid + cells, m.colsum,
                     nx, ny);
  pe.mark(9, st);
  pe.mark(10, st);
  gemm_dct_rows(m, st, mid, outc, 2 * ny, true);
  const int sn = (int)(level % 3), snew = (int)((level + 1) % 3);
  hipLaunchKernelGGL(k_gemm_finalize, dim3(ny), dim3(GEMM_THREADS), 0, st, outc, m.phi[sn],
                     m.psi[sn], m.colsum, m.phi[snew], m.psi[snew], nx, ny);
  pe.mark(11, st);
  return CCMSAV_OK;
}

int periodic_solve_pc(const Member& m, int precision, hipStream_t st, const double* rhs,
                      double* out_chi, double* out_zeta, const PerConst& pc);

// One step of the single member with periodic boundaries (FP64): the stencil
// pass with wrap-around ghosts, the seven elliptic solves of Algorithm 1 by
// the FFT solver (chi^{-1} f_lin, zeta^{-1} g_lin and zeta^{-1} L~ in place,
// chi^{-1} of S~, H, Q~, K~ into psol), the inner products of App. B Step 4
// in physical space, the 5x5 solve, and the combination into level n+1.
int enqueue_step_periodic(ccmsav_ctx* c, int64_t level, hipStream_t st, PhaseEvents pe) {
  const Member& m = c->mem[0];
  const SizeClass& k = c->cls[0];
  const int t = table_of_level(level);
  const MemberArgs* tab = c->d_args + (size_t)t * c->mem.size();
  const StepConst& sc = c->h_args[(size_t)t * c->mem.size()].k;
  const int nx = m.p.nx, ny = m.p.ny;
  const size_t cells = (size_t)nx * ny;
  double* rm = static_cast<double*>(m.rm);
  auto field = [&](int f) { return rm + (size_t)f * cells; };
  const PerConst pc{sc.C1, sc.C2, sc.C3, sc.alpha, sc.lam, m.p.h};
  pe.mark(0, st);
  hipLaunchKernelGGL(k_stencil<double>, dim3(stencil_grid(c, true, k.sh.blocks)),
                     dim3(STENCIL_THREADS), 0, st, tab, k.d_idx, k.sh.blocks, k.sh.blocks);
  pe.mark(1, st);
  pe.mark(2, st);
  int r = periodic_solve_pc(m, c->precision, st, field(M_F), field(M_F), nullptr, pc);
  const int chi_src[4] = {M_S, M_H, M_Q, M_K};
  for (int i = 0; i < 4 && r == CCMSAV_OK; ++i)
    r = periodic_solve_pc(m, c->precision, st, field(chi_src[i]), m.psol + (size_t)i * cells,
                          nullptr, pc);
  if (r == CCMSAV_OK)
    r = periodic_solve_pc(m, c->precision, st, field(M_G), nullptr, field(M_G), pc);
  if (r == CCMSAV_OK)
    r = periodic_solve_pc(m, c->precision, st, field(M_L), nullptr, field(M_L), pc);
  if (r != CCMSAV_OK) return r;
  pe.mark(3, st);
  pe.mark(4, st);
  hipLaunchKernelGGL(k_per_gram, dim3(ny), dim3(PER_THREADS), 0, st, rm, m.psol, m.part2, nx, ny);
  pe.mark(5, st);
  pe.mark(6, st);
  launch_solve(st, k, 1, tab);
  pe.mark(7, st);
  pe.mark(8, st);
  const int snew = (int)((level + 1) % 3);
  const int blocks = (int)std::min<size_t>((cells + PER_THREADS - 1) / PER_THREADS, 8192);
  hipLaunchKernelGGL(k_per_combine, dim3(blocks), dim3(PER_THREADS), 0, st, rm, m.psol,
                     m.ds->coef, m.phi[snew], m.psi[snew], cells);
  pe.mark(9, st);
  pe.mark(10, st);
  pe.mark(11, st);
  return hipGetLastError() == hipSuccess ? CCMSAV_OK : CCMSAV_EHIP;
}

// The whole step as one launch of the persistent kernel (all members, all
// passes); the step is reported as phase 0 of the per-phase timing.
int enqueue_step_persistent(ccmsav_ctx* c, int64_t level, hipStream_t st, PhaseEvents pe) {
  const MemberArgs* tab = c->d_args + (size_t)table_of_level(level) * c->mem.size();
  pe.mark(0, st);
  hipLaunchKernelGGL(k_persist_step<float>, dim3(c->ps_grid), dim3(PS_THREADS), 0, st,
                     c->ps_plan, tab, c->bar, c->spin_limit);
  for (int i = 1; i < 2 * kNumPhases; ++i) pe.mark(i, st);
  return CCMSAV_OK;
}

// Work list and grid of the persistent launch: per pass and size class, the
// groups of virtual blocks one workgroup runs at once (PS_THREADS / threads
// of the body), and as many workgroups as the device holds at once.
int build_persist_plan(ccmsav_ctx* c) {
  static_assert(STENCIL_THREADS == PS_THREADS && SOLVE_THREADS_SMALL == PS_THREADS,
                "one stencil band and one 5x5 system per workgroup");
  if (c->cls.size() > (size_t)PS_MAX_CLASSES) return CCMSAV_EUNSUPPORTED;
  PersistPlan& pl = c->ps_plan;
  pl = PersistPlan{};
  pl.ncls = (int)c->cls.size();
  for (size_t ki = 0; ki < c->cls.size(); ++ki) {
    const SizeClass& k = c->cls[ki];
    // every member of the class takes the 256-thread 5x5 kernel in both paths
    if (solve_threads((size_t)1 << (k.lx + k.ly)) != SOLVE_THREADS_SMALL) return CCMSAV_EUNSUPPORTED;
    pl.cls[ki] = PersistClass{k.lx, k.ly, k.count, k.d_idx, k.sh.blocks};
    const int nx = 1 << k.lx, ny = 1 << k.ly;
    for (int ph = 0; ph < PS_PHASES; ++ph) {
      const int n = (ph == 1 || ph == 5) ? nx : ny;
      const int nt = ps_body_threads<float>(ph, n);
      if (nt > PS_THREADS || PS_THREADS % nt != 0) return CCMSAV_EUNSUPPORTED;
      const int g = PS_THREADS / nt;
      const long total = (long)k.count * ps_blocks_per_member<float>(ph, nx, ny, k.sh.blocks);
      if (total % g != 0) return CCMSAV_EUNSUPPORTED;
      pl.off[ph][ki + 1] = pl.off[ph][ki] + (int)(total / g);
    }
  }
  int dev = 0, cus = 0, per_cu = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu, reinterpret_cast<const void*>(k_persist_step<float>), PS_THREADS, 0));
  if (per_cu < 1 || cus < 1) return CCMSAV_EUNSUPPORTED;
  c->ps_grid = per_cu * cus;
  return CCMSAV_OK;
}

int enqueue_step_level(ccmsav_ctx* c, int64_t level, hipStream_t st,
                       PhaseEvents pe = PhaseEvents{nullptr}, int only = -1) {
  if (is_gemm(c->precision)) return enqueue_step_gemm(c, level, st, pe);
  if (c->periodic) return enqueue_step_periodic(c, level, st, pe);
  if (c->persistent) return enqueue_step_persistent(c, level, st, pe);
  const int t = table_of_level(level);
  Tuner tu;
  if (!c->tuned) {
    tu.on = true;
    tu.ev.resize(c->cls.size() * kNumTuned * kNumVariants * kTuneReps * 2, nullptr);
    for (hipEvent_t& e : tu.ev)
      if (hipEventCreate(&e) != hipSuccess) return CCMSAV_EHIP;
  }
  if (c->precision == CCMSAV_MIXED)
    enqueue_step_kind<float>(c, t, st, pe, tu, only);
  else
    enqueue_step_kind<double>(c, t, st, pe, tu, only);
  if (tu.on) {
    int rc = hipStreamSynchronize(st) == hipSuccess ? CCMSAV_OK : CCMSAV_EHIP;
    for (size_t ki = 0; ki < c->cls.size() && rc == CCMSAV_OK; ++ki)
      for (int tk = 0; tk < kNumTuned; ++tk) {
        int best = 0;
        for (int v = 0; v < kNumVariants; ++v) {
          float mn = 1e30f;
          for (int r = 0; r < kTuneReps; ++r) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, tu.ev[tu.at(ki, tk, v, r, 0)],
                                    tu.ev[tu.at(ki, tk, v, r, 1)]) != hipSuccess)
              rc = CCMSAV_EHIP;
            mn = std::min(mn, ms);
          }
          c->cls[ki].tune_ms[tk][v] = mn;
          if (mn < c->cls[ki].tune_ms[tk][best]) best = v;
        }
        c->cls[ki].var[tk] = best;
      }
    for (hipEvent_t e : tu.ev)
      if (e) (void)hipEventDestroy(e);
    if (rc != CCMSAV_OK) return rc;
    c->tuned = true;
  }
  return CCMSAV_OK;
}

// Capture three steady-state steps (levels 3k, 3k+1, 3k+2, k >= 1) into a graph.
// Size classes are independent (members share no data), so with several of
// them each class's three steps form their own branch of the graph, forked
// from and joined to the capture stream, and the device runs the branches
// side by side.
int capture_graph(ccmsav_ctx* c) {
  if (c->gexec) return CCMSAV_OK;
  // one branch per size class (the persistent launch covers them all)
  const size_t nb = (c->cls.size() > 1 && !c->persistent) ? c->cls.size() - 1 : 0;
  while (c->bstream.size() < nb) {
    hipStream_t s = nullptr;
    hipEvent_t e = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    c->bstream.push_back(s);
    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    c->bevent.push_back(e);
  }
  if (nb > 0 && !c->ev_fork) HIP_TRY(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
  HIP_TRY(hipStreamBeginCapture(c->gstream, hipStreamCaptureModeRelaxed));
  bool ok = true;   // the capture is ended whatever happens inside it
  if (nb == 0) {
    for (int64_t lv = 3; lv < 6; ++lv) ok &= enqueue_step_level(c, lv, c->gstream) == CCMSAV_OK;
  } else {
    ok &= hipEventRecord(c->ev_fork, c->gstream) == hipSuccess;
    for (size_t i = 0; i < nb && ok; ++i) {
      ok &= hipStreamWaitEvent(c->bstream[i], c->ev_fork, 0) == hipSuccess;
      for (int64_t lv = 3; lv < 6; ++lv)
        ok &= enqueue_step_level(c, lv, c->bstream[i], PhaseEvents{nullptr}, (int)i + 1) ==
              CCMSAV_OK;
      ok &= hipEventRecord(c->bevent[i], c->bstream[i]) == hipSuccess;
    }
    for (int64_t lv = 3; lv < 6; ++lv)
      ok &= enqueue_step_level(c, lv, c->gstream, PhaseEvents{nullptr}, 0) == CCMSAV_OK;
    for (size_t i = 0; i < nb; ++i)
      ok &= hipStreamWaitEvent(c->gstream, c->bevent[i], 0) == hipSuccess;
  }
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(c->gstream, &g);
  if (!ok || e != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return CCMSAV_EHIP;
  }
  const hipError_t ei = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) {
    c->gexec = nullptr;
    return CCMSAV_EHIP;
  }
  return CCMSAV_OK;
}

int read_err_member(ccmsav_ctx* c, int m, int* err) {
  *err = 0;
  GridBarrier b{};
  HIP_TRY(hipMemcpyAsync(err, &c->mem[m].ds->err, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  if (c->persistent && c->bar)
    HIP_TRY(hipMemcpyAsync(&b, c->bar, sizeof(b), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (b.err) *err |= ERR_BARRIER;
  return CCMSAV_OK;
}

int read_err(ccmsav_ctx* c, int* err) {
  *err = 0;
  std::vector<int> e(c->mem.size(), 0);
  GridBarrier b{};
  for (size_t m = 0; m < c->mem.size(); ++m)
    HIP_TRY(hipMemcpyAsync(&e[m], &c->mem[m].ds->err, sizeof(int), hipMemcpyDeviceToHost,
                           c->stream));
  if (c->persistent)
    HIP_TRY(hipMemcpyAsync(&b, c->bar, sizeof(b), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (int v : e) *err |= v;
  if (b.err) *err |= ERR_BARRIER;
  return CCMSAV_OK;
}

void free_ctx(ccmsav_ctx* c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->ev_in) (void)hipEventDestroy(c->ev_in);
  if (c->ev_out) (void)hipEventDestroy(c->ev_out);
  if (c->gstream) (void)hipStreamDestroy(c->gstream);
  for (hipStream_t b : c->bstream) (void)hipStreamDestroy(b);
  for (hipEvent_t e : c->bevent) (void)hipEventDestroy(e);
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->owns_ws && c->ws) (void)hipFree(c->ws);
  delete c;
}

int run_diag(ccmsav_ctx* c, int mi, bool energy) {
  const Member& m = c->mem[mi];
  const int64_t n = c->level;
  const int sn = (int)(n % 3), sm = (int)((n + 2) % 3), smm = (int)((n + 1) % 3);
  DiagConst d = make_diag(m.p);
  d.with_d = (energy && n >= 2) ? 1 : 0;
  const double* p1 = m.phi[sn];
  const double* p0 = n >= 1 ? m.phi[sm] : p1;
  const double* pm = n >= 2 ? m.phi[smm] : p0;
  const double* s1 = m.psi[sn];
  const double* s0 = n >= 1 ? m.psi[sm] : s1;
  const double* sm_ = n >= 2 ? m.psi[smm] : s0;
  hipLaunchKernelGGL(k_energy_sums, dim3(m.p.ny), dim3(DIAG_THREADS), 0, c->stream, p1, p0, pm,
                     s1, s0, sm_, m.parte, m.p.nx, m.p.ny, d);
  hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(DIAG_THREADS), 0, c->stream, m.parte, m.p.ny,
                     m.ds, sn, n >= 1 ? sm : sn, d);
  if (hipGetLastError() != hipSuccess) return CCMSAV_EHIP;
  return CCMSAV_OK;
}

// FP32 -> bfloat16 on the host, round to nearest even (finite inputs).
uint16_t host_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, sizeof(u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
float host_bf16_to_f32(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, sizeof(f));
  return f;
}

// Orthonormal DCT-II matrix of size n (App. C), D(k, i) = s_k cos(pi k (2i + 1) / (2n)),
// and its transpose, row-major, each as three bf16 parts (hi, mid, lo) at
// out + {0, 1, 2} n^2 (D) and out + {3, 4, 5} n^2 (D^T).
int upload_dct_matrix(uint16_t* out, int n, hipStream_t st, MfMat& d, MfMat& dt) {
  const size_t nn = (size_t)n * n;
  std::vector<uint16_t> h(6 * nn);
  const double s0 = std::sqrt(1.0 / n), s1 = std::sqrt(2.0 / n);
  for (int k = 0; k < n; ++k)
    for (int i = 0; i < n; ++i) {
      double v = (k == 0 ? s0 : s1) * std::cos(M_PI * k * (2.0 * i + 1.0) / (2.0 * n));
      for (int q = 0; q < 3; ++q) {
        const uint16_t b = host_bf16((float)v);
        h[q * nn + (size_t)k * n + i] = b;
        h[(3 + q) * nn + (size_t)i * n + k] = b;
        v -= (double)host_bf16_to_f32(b);
      }
    }
  d = MfMat{{out, out + nn, out + 2 * nn}};
  dt = MfMat{{out + 3 * nn, out + 4 * nn, out + 5 * nn}};
  const bool ok =
      hipMemcpyAsync(out, h.data(), h.size() * sizeof(uint16_t), hipMemcpyHostToDevice, st) ==
      hipSuccess;
  // the host table must outlive the copy, also when it failed
  if (hipStreamSynchronize(st) != hipSuccess || !ok) return CCMSAV_EHIP;
  return CCMSAV_OK;
}

// The matrices and tables of the factored transform of n1 n2 points (FsMats),
// built in FP64: each matrix as three bf16 parts at out (the matrices one
// after another, each as hi, mid, lo), the two tables as float2 behind them.
int upload_fs_matrices(void* out, int n1, int n2, hipStream_t st, FsMats& f) {
  const int n = n1 * n2;
  const size_t e1 = 2 * (size_t)n1 * n1, e2 = 2 * (size_t)n2 * n2, e3 = 4 * (size_t)n1 * n1,
               e4 = 2 * (size_t)n2 * n2;
  const size_t o1 = 0, o2 = 3 * e1, o3 = o2 + 3 * e2, o4 = o3 + 3 * e3;
  const size_t tab = fs_table_offset(n1, n2);
  std::vector<uint8_t> h(tab + 2 * (size_t)n * sizeof(float2), 0);
  uint16_t* hm = reinterpret_cast<uint16_t*>(h.data());
  // v = hi + mid + lo, each part the bf16 rounding of what the earlier leave
  auto put = [&](size_t off, size_t e, size_t idx, double v) {
    for (int q = 0; q < 3; ++q) {
      const uint16_t b = host_bf16((float)v);
      hm[off + q * e + idx] = b;
      v -= (double)host_bf16_to_f32(b);
    }
  };
  // exp(-i pi num / den) as (c, s), num reduced mod 2 den first
  auto ex = [](long num, long den, double& c, double& sn) {
    const double a = M_PI * (double)(num % (2 * den)) / (double)den;
    c = std::cos(a);
    sn = -std::sin(a);
  };
  const double up = std::sqrt(0.5 * n), down = std::sqrt(2.0 / n);
  double c, sn;
  for (int k = 0; k < n1; ++k)
    for (int j = 0; j < n1; ++j) {
      ex(2L * j * k, n1, c, sn);               // W_N1^(jk)
      put(o1, e1, (size_t)(2 * k) * n1 + j, c);
      put(o1, e1, (size_t)(2 * k + 1) * n1 + j, sn);
      ex((long)j * (4 * k + 1), 2L * n1, c, sn);
      c *= up;
      sn *= up;
      const size_t w = 2 * (size_t)n1;
      put(o3, e3, (size_t)(2 * k) * w + j, c);
      put(o3, e3, (size_t)(2 * k) * w + n1 + j, -sn);
      put(o3, e3, (size_t)(2 * k + 1) * w + j, sn);
      put(o3, e3, (size_t)(2 * k + 1) * w + n1 + j, c);
    }
  for (int k = 0; k < n2; ++k)
    for (int j = 0; j < n2; ++j) {
      const size_t w = 2 * (size_t)n2;
      ex((long)k * (4 * j + 1), 2L * n2, c, sn);
      put(o2, e2, (size_t)k * w + j, down * c);
      put(o2, e2, (size_t)k * w + n2 + j, -down * sn);
      ex(2L * j * k, n2, c, sn);               // W_N2^(jk)
      put(o4, e4, (size_t)k * w + j, c / n);
      put(o4, e4, (size_t)k * w + n2 + j, -sn / n);
    }
  float2* tw = reinterpret_cast<float2*>(h.data() + tab);
  for (int k1 = 0; k1 < n1; ++k1)
    for (int j = 0; j < n2; ++j) {
      ex((long)k1 * (4 * j + 1), 2L * n, c, sn);
      tw[(size_t)k1 * n2 + j] = make_float2((float)c, (float)sn);
      ex((long)j * (4 * k1 + 1), 2L * n, c, sn);
      tw[(size_t)n + (size_t)k1 * n2 + j] = make_float2((float)c, (float)sn);
    }
  const uint16_t* dm = static_cast<const uint16_t*>(out);
  auto mat = [&](size_t off, size_t e) { return MfMat{{dm + off, dm + off + e, dm + off + 2 * e}}; };
  f.l1 = log2_exact(n1);
  f.l2 = log2_exact(n2);
  f.d1 = mat(o1, e1);
  f.d2 = mat(o2, e2);
  f.d1i = mat(o3, e3);
  f.d2i = mat(o4, e4);
  f.twf = reinterpret_cast<const float2*>(static_cast<const char*>(out) + tab);
  f.twi = f.twf + n;
  const bool ok =
      hipMemcpyAsync(out, h.data(), h.size(), hipMemcpyHostToDevice, st) == hipSuccess;
  // the host table must outlive the copy, also when it failed
  if (hipStreamSynchronize(st) != hipSuccess || !ok) return CCMSAV_EHIP;
  return CCMSAV_OK;
}

bool valid_member(const ccmsav_ctx* c, int32_t member) {
  return c && member >= 0 && member < (int32_t)c->mem.size();
}

const char* kStatusText[] = {
    "success",
    "invalid argument or parameter",
    "out of memory or workspace too small",
    "HIP runtime error",
    "domain error (vanishing SAV normaliser, singular 5x5 system or non-positive mobility)",
    "non-finite value in the state",
    "unsupported grid size or precision mode",
    "an iterative solve did not reach its tolerance",
    "a grid barrier of the persistent launch failed",
};

}  // namespace

namespace {

// Launches of the periodic solver over the line length (16 .. 4096).
constexpr int kPerMaxLog = 12;
struct PerLaunch {
  using Rows = void (*)(hipStream_t, int, const double*, cpx<double>*, int, size_t);
  using Cols = void (*)(hipStream_t, int, const cpx<double>*, cpx<double>*, cpx<double>*, int,
                        size_t, PerConst);
  using Inv = void (*)(hipStream_t, int, const cpx<double>*, double*, int, size_t);
  template <int N>
  static void rows(hipStream_t st, int grid, const double* rhs, cpx<double>* col, int ny,
                   size_t cs) {
    hipLaunchKernelGGL(k_per_rows<N>, dim3(grid), dim3(line_threads(N)), 0, st, rhs, col, ny, cs);
  }
  template <int N>
  static void cols(hipStream_t st, int grid, const cpx<double>* col, cpx<double>* oc,
                   cpx<double>* oz, int nx, size_t cs, PerConst k) {
    hipLaunchKernelGGL(k_per_cols<N>, dim3(grid), dim3(line_threads(N)), 0, st, col, oc, oz, nx,
                       cs, k);
  }
  template <int N>
  static void inv(hipStream_t st, int grid, const cpx<double>* col, double* out, int ny,
                  size_t cs) {
    hipLaunchKernelGGL(k_per_rows_inv<N>, dim3(grid), dim3(line_threads(N)), 0, st, col, out, ny,
                       cs);
  }
  template <int... L> struct Tables {
    static constexpr Rows t_rows[] = {&rows<(1 << L)>...};
    static constexpr Cols t_cols[] = {&cols<(1 << L)>...};
    static constexpr Inv t_inv[] = {&inv<(1 << L)>...};
  };
  using T = Tables<4, 5, 6, 7, 8, 9, 10, 11, 12>;
};

// Periodic chi^{-1} rhs and zeta^{-1} rhs of member m (FP64 transforms) with
// the operator constants pc, on stream st, with three column buffers of
// (nx/2 + 1) columns in the member's intermediate region. An output may be
// rhs itself (the row pass has read rhs before the inverse rows write).
int periodic_solve_pc(const Member& m, int precision, hipStream_t st, const double* rhs,
                      double* out_chi, double* out_zeta, const PerConst& pc) {
  const int nx = m.p.nx, ny = m.p.ny;
  if (m.lx > kPerMaxLog || m.ly > kPerMaxLog) return CCMSAV_EUNSUPPORTED;
  const size_t cs = (size_t)ny + 66;             // column stride, off a power of two
  const size_t colb = (size_t)(nx / 2 + 1) * cs;
  const size_t need = 3 * colb * sizeof(cpx<double>);
  const size_t have = M_NFIELD * strip_field(nx, ny, (int)mid_elem(precision)) *
                      mid_elem(precision);
  if (need > have) return CCMSAV_EUNSUPPORTED;
  cpx<double>* col = static_cast<cpx<double>*>(m.mid);
  cpx<double>* cc = col + colb;
  cpx<double>* cz = cc + colb;
  using PT = PerLaunch::T;
  PT::t_rows[m.lx - kMinLog](st, ny / 2, rhs, col, ny, cs);
  PT::t_cols[m.ly - kMinLog](st, nx / 2 + 1, col, out_chi ? cc : nullptr,
                             out_zeta ? cz : nullptr, nx, cs, pc);
  if (out_chi) PT::t_inv[m.lx - kMinLog](st, ny / 2, cc, out_chi, ny, cs);
  if (out_zeta) PT::t_inv[m.lx - kMinLog](st, ny / 2, cz, out_zeta, ny, cs);
  return hipGetLastError() == hipSuccess ? CCMSAV_OK : CCMSAV_EHIP;
}

// The standalone periodic solve of member 0 with the BDF2 operators.
int periodic_solve(ccmsav_ctx* c, const double* rhs, double* out_chi, double* out_zeta) {
  const StepConst& k = c->h_args[(size_t)kSolveTable * c->mem.size()].k;
  const PerConst pc{k.C1, k.C2, k.C3, k.alpha, k.lam, c->mem[0].p.h};
  return periodic_solve_pc(c->mem[0], c->precision, c->stream, rhs, out_chi, out_zeta, pc);
}

// Upload `a` (a copy of the standalone-solve table entry, with the operator
// constants to use) as that entry, with the outputs of member 0's solve: an
// output that is not requested goes to intermediate slots 2-3, which the
// solve does not read.
int set_solve_args(ccmsav_ctx* c, MemberArgs a, double* out_chi, double* out_zeta) {
  const Member& m = c->mem[0];
  const size_t me = mid_elem(c->precision);
  double* tmp = reinterpret_cast<double*>(static_cast<char*>(m.mid) +
                                          2 * strip_field(m.p.nx, m.p.ny, (int)me) * me);
  a.phi_new = to_global(out_chi ? out_chi : tmp);
  a.psi_new = to_global(out_zeta ? out_zeta : tmp);
  MemberArgs* d = c->d_args + (size_t)kSolveTable * c->mem.size();
  HIP_TRY(hipMemcpyAsync(d, &a, sizeof(MemberArgs), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return CCMSAV_OK;
}

// chi^{-1} rhs and zeta^{-1} rhs of member 0 with the uploaded solve entry,
// on the context's stream: row DCT-II, column solve, row DCT-III.
void launch_solve(ccmsav_ctx* c, const double* rhs) {
  const Member& m = c->mem[0];
  const MemberArgs* d = c->d_args + (size_t)kSolveTable * c->mem.size();
  const SizeClass& k = c->cls[0];
  auto run = [&](auto tm) {
    using TM = decltype(tm);
    using LT = typename Launch<TM>::T;
    LT::t_rd[m.lx - kMinLog](c->stream, m.p.ny, rhs, static_cast<TM*>(m.mid), M_F, m.p.ny,
                             nullptr);
    LT::t_col_solve[k.var[TUNE_COL_SOLVE]][m.ly - kMinLog](c->stream, m.p.nx,
                                                           Batch{d, k.d_idx, m.p.nx});
    const int vi = k.var[TUNE_ROW_IDCT];
    const int per = m.p.ny / row_idct_rows<TM>(m.p.nx, vi);
    LT::t_row_idct[vi][m.lx - kMinLog](c->stream, per, Batch{d, k.d_idx, per});
  };
  if (c->precision != CCMSAV_FP64)
    run(0.0f);
  else
    run(0.0);
}

// ---- allocation-free standalone solve ------------------------------------------

// Largest grid of ccmsav_elliptic_solve_noalloc: 1024 cells per direction.
constexpr int kNoallocMaxLog = 10;
constexpr int kNoallocMaxN = 1 << kNoallocMaxLog;
// Scratch of one call, sized for FP64 intermediates at the largest grid:
// the row-transformed right-hand side (one strip-major field, which also
// takes an output that is not requested once the column solve has read it),
// the two column-solved fields, the two eigenvalue tables, the unit
// combination weights, the argument block and the member index.
constexpr size_t kNoallocField = strip_field(kNoallocMaxN, kNoallocMaxN, 8) * 8;
constexpr size_t kNoallocLayout =
    align_up_c(kNoallocField) + align_up_c(2 * kNoallocField) + 2 * align_up_c(kNoallocMaxN * 8) +
    align_up_c(8 * sizeof(double)) + align_up_c(sizeof(MemberArgs)) + align_up_c(sizeof(int));
static_assert(kNoallocLayout <= CCMSAV_NOALLOC_SCRATCH_BYTES, "scratch layout exceeds its size");
static_assert(sizeof(MemberArgs) % sizeof(uint64_t) == 0, "argument block copied as 8-byte words");

// Operator tables, unit weights, argument block and member index of one
// allocation-free solve, written on the device (no host-to-device copy).
__global__ void __launch_bounds__(256)
k_noalloc_setup(MemberArgs a, gptr<MemberArgs> args, gptr<int> idx, gptr<double> lamx,
                gptr<double> lamy, gptr<double> coef, int nx, int ny, double h) {
  const int tid = threadIdx.x;
  // Eigenvalues of -Delta_h per direction (App. C): (4/h^2) sin^2(pi k / (2 n)).
  for (int k = tid; k < nx; k += blockDim.x) {
    const double s = sin(M_PI * k / (2.0 * nx));
    lamx[k] = 4.0 / (h * h) * s * s;
  }
  for (int k = tid; k < ny; k += blockDim.x) {
    const double s = sin(M_PI * k / (2.0 * ny));
    lamy[k] = 4.0 / (h * h) * s * s;
  }
  if (tid < 8) coef[tid] = (tid == 0 || tid == 5) ? 1.0 : 0.0;
  const uint64_t* src = reinterpret_cast<const uint64_t*>(&a);
  const auto dst = reinterpret_cast<gptr<uint64_t>>(args);
  for (int i = tid; i < (int)(sizeof(MemberArgs) / sizeof(uint64_t)); i += blockDim.x)
    dst[i] = src[i];
  if (tid == 0) idx[0] = 0;
}

// Device address of the scratch array on each device, looked up once per
// device with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch[kMaxDevices] = {};

// Whether p is device (or managed) memory of device dev.
bool on_device(const void* p, int dev) {
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();     // clear the error this query leaves for a host pointer
    return false;
  }
  return (at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged) && at.device == dev;
}

}  // namespace

// Scratch memory of ccmsav_elliptic_solve_noalloc: a fixed array on every
// GPU the library runs on, held until the process ends. Host code never
// uses this name as an address; it uses the device address looked up per
// device (noalloc_scratch).
static __device__ __align__(256) unsigned char scratch[CCMSAV_NOALLOC_SCRATCH_BYTES];

namespace {

// Device address of `scratch` on the current device (set up at the first
// call on that device), or nullptr with *rc set.
char* noalloc_scratch(int* rc) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) {
    *rc = CCMSAV_EHIP;
    return nullptr;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    *rc = CCMSAV_EUNSUPPORTED;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      *rc = CCMSAV_EHIP;
      return nullptr;
    }
    g_scratch[dev] = static_cast<char*>(ptr);
  }
  *rc = CCMSAV_OK;
  return g_scratch[dev];
}

}  // namespace

extern "C" {

size_t ccmsav_workspace_bytes_batch(int32_t nmemb, const ccmsav_params* p) {
  if (check_batch(nmemb, p) != CCMSAV_OK) return 0;
  return batch_layout(nmemb, p).total;
}

size_t ccmsav_workspace_bytes(const ccmsav_params* p) {
  return ccmsav_workspace_bytes_batch(1, p);
}

int ccmsav_init_batch(ccmsav_ctx** out, int32_t nmemb, const ccmsav_params* p,
                      const double* const* phi0, const double* const* psi0, void* workspace,
                      size_t ws_bytes, void* hip_stream) {
  if (!out || !phi0 || !psi0) return CCMSAV_EINVAL;
  *out = nullptr;
  const int pc = check_batch(nmemb, p);
  if (pc != CCMSAV_OK) return pc;
  for (int32_t m = 0; m < nmemb; ++m)
    if (!phi0[m] || !psi0[m]) return CCMSAV_EINVAL;
  const BatchLayout BL = batch_layout(nmemb, p);
  if (workspace && ws_bytes < BL.total) return CCMSAV_ENOMEM;
  if (workspace && (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0) return CCMSAV_EINVAL;
  ccmsav_ctx* c = new (std::nothrow) ccmsav_ctx();
  if (!c) return CCMSAV_ENOMEM;
  c->precision = p[0].precision;
  c->graph = (p[0].flags & CCMSAV_FLAG_GRAPH) != 0;
  c->bdf1 = (p[0].flags & CCMSAV_FLAG_BDF1) != 0;
  c->periodic = is_periodic(&p[0]);
  c->classical = is_classical(&p[0]);
  c->persistent = is_persistent(&p[0]);
  // the periodic step has no launch variants, the persistent one fixed ones
  c->tuned = c->periodic || c->persistent;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->owns_ws = workspace == nullptr;
  if (c->owns_ws) {
    if (hipMalloc(&c->ws, BL.total) != hipSuccess) {
      c->ws = nullptr;
      free_ctx(c);
      return CCMSAV_ENOMEM;
    }
    c->ws_bytes = BL.total;
  } else {
    c->ws = workspace;
    c->ws_bytes = ws_bytes;
  }
  char* base = static_cast<char*>(c->ws);
  c->d_args = reinterpret_cast<MemberArgs*>(base + BL.args);
  int* d_idx = reinterpret_cast<int*>(base + BL.idx);
  c->bar = reinterpret_cast<GridBarrier*>(base + BL.bar);
  auto fail = [&](int code) {
    (void)hipStreamSynchronize(c->stream);
    free_ctx(c);
    return code;
  };
  // the barrier state is read by every status check, the first ones below
  if (hipMemsetAsync(c->bar, 0, sizeof(GridBarrier), c->stream) != hipSuccess)
    return fail(CCMSAV_EHIP);

  c->mem.resize(nmemb);
  for (int32_t mi = 0; mi < nmemb; ++mi) {
    Member& m = c->mem[mi];
    m.p = p[mi];
    m.lx = log2_exact(m.p.nx);
    m.ly = log2_exact(m.p.ny);
    m.sh = stencil_shape(m.p.nx, m.p.ny);
    const Layout L = layout(&m.p);
    char* mb = base + BL.member[mi];
    const size_t cells = (size_t)m.p.nx * m.p.ny;
    double* st = reinterpret_cast<double*>(mb + L.state);
    for (int s = 0; s < 3; ++s) {
      m.phi[s] = st + (size_t)(2 * s) * cells;
      m.psi[s] = st + (size_t)(2 * s + 1) * cells;
    }
    m.rm = mb + L.rm;
    m.mid = mb + L.mid;
    m.outc = mb + L.outc;
    m.part1 = reinterpret_cast<double*>(mb + L.part1);
    m.part2 = reinterpret_cast<double*>(mb + L.part2);
    m.parte = reinterpret_cast<double*>(mb + L.parte);
    m.lamx = reinterpret_cast<double*>(mb + L.lamx);
    m.lamy = reinterpret_cast<double*>(mb + L.lamy);
    m.colsum = reinterpret_cast<double*>(mb + L.colsum);
    m.unit_coef = reinterpret_cast<double*>(mb + L.unit);
    m.ds = reinterpret_cast<DevScalars*>(mb + L.ds);
    m.psol = is_periodic(&m.p) ? reinterpret_cast<double*>(mb + L.psol) : nullptr;
    if (is_classical(&m.p)) {
      double* f = reinterpret_cast<double*>(mb + L.cl);
      m.cl_x = f;
      m.cl_r = f + 2 * cells;
      m.cl_p[0] = f + 4 * cells;
      m.cl_p[1] = f + 6 * cells;
      m.cl_q = f + 8 * cells;
      m.cl_z = f + 10 * cells;
      m.mob_e = f + 12 * cells;
      m.mob_n = f + 13 * cells;
      m.cl_part = reinterpret_cast<double*>(mb + L.clpart);
      m.cl_sc = reinterpret_cast<PcgScalars*>(mb + L.clsc);
    }
    if (is_gemm(m.p.precision)) {
      // per direction: the factored transform's DFT matrices, or D and D^T
      auto setup = [&](int n, size_t off, FsMats& f, MfMat& d, MfMat& dt) {
        d = dt = MfMat{{nullptr, nullptr, nullptr}};
        if (const int n1 = fs_n1(n)) return upload_fs_matrices(mb + off, n1, n / n1, c->stream, f);
        return upload_dct_matrix(reinterpret_cast<uint16_t*>(mb + off), n, c->stream, d, dt);
      };
      if (setup(m.p.nx, L.dx, m.fsx, m.dx, m.dxt) != CCMSAV_OK ||
          setup(m.p.ny, L.dy, m.fsy, m.dy, m.dyt) != CCMSAV_OK)
        return fail(CCMSAV_EHIP);
      m.fs_w = uses_fs(&m.p) ? reinterpret_cast<float*>(mb + L.fs) : nullptr;
    }

    // Eigenvalues of -Delta_h per direction (App. C): (4/h^2) sin^2(pi k / (2 n)).
    std::vector<double> lx(m.p.nx), ly(m.p.ny);
    for (int k = 0; k < m.p.nx; ++k) {
      const double s = std::sin(M_PI * k / (2.0 * m.p.nx));
      lx[k] = 4.0 / (m.p.h * m.p.h) * s * s;
    }
    for (int k = 0; k < m.p.ny; ++k) {
      const double s = std::sin(M_PI * k / (2.0 * m.p.ny));
      ly[k] = 4.0 / (m.p.h * m.p.h) * s * s;
    }
    const double unit[8] = {1.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0};
    bool ok = hipMemcpyAsync(m.lamx, lx.data(), m.p.nx * sizeof(double), hipMemcpyHostToDevice,
                             c->stream) == hipSuccess &&
              hipMemcpyAsync(m.lamy, ly.data(), m.p.ny * sizeof(double), hipMemcpyHostToDevice,
                             c->stream) == hipSuccess &&
              hipMemcpyAsync(m.unit_coef, unit, sizeof(unit), hipMemcpyHostToDevice,
                             c->stream) == hipSuccess &&
              hipMemsetAsync(m.ds, 0, sizeof(DevScalars), c->stream) == hipSuccess &&
              hipMemcpyAsync(m.phi[0], phi0[mi], cells * sizeof(double), hipMemcpyDefault,
                             c->stream) == hipSuccess &&
              hipMemcpyAsync(m.psi[0], psi0[mi], cells * sizeof(double), hipMemcpyDefault,
                             c->stream) == hipSuccess;
    // the host tables must outlive the copies, also when one of them failed
    if (hipStreamSynchronize(c->stream) != hipSuccess || !ok) return fail(CCMSAV_EHIP);
    const DiagConst d = make_diag(m.p);
    hipLaunchKernelGGL(k_init_sums, dim3(m.p.ny), dim3(DIAG_THREADS), 0, c->stream, m.phi[0],
                       m.psi[0], m.parte, m.p.nx, m.p.ny, d);
    hipLaunchKernelGGL(k_init_final, dim3(1), dim3(DIAG_THREADS), 0, c->stream, m.parte, m.p.ny,
                       m.ds, d);
    if (hipGetLastError() != hipSuccess) return fail(CCMSAV_EHIP);
  }
  // Arc-length targets and the status of the initial reductions.
  for (int32_t mi = 0; mi < nmemb; ++mi) {
    Member& m = c->mem[mi];
    double A = 0.0;
    int err = 0;
    if (hipMemcpyAsync(&A, &m.ds->totals[0], sizeof(double), hipMemcpyDeviceToHost, c->stream) !=
            hipSuccess ||
        read_err_member(c, mi, &err) != CCMSAV_OK)
      return fail(CCMSAV_EHIP);
    m.p.A = A;
    const int st0 = status_from_err(err);
    if (st0 != CCMSAV_OK) return fail(st0);
  }

  // Size classes and their member lists.
  std::vector<int> order;
  for (int32_t mi = 0; mi < nmemb; ++mi) {
    bool seen = false;
    for (const SizeClass& k : c->cls) seen = seen || (k.lx == c->mem[mi].lx && k.ly == c->mem[mi].ly);
    if (seen) continue;
    SizeClass k{c->mem[mi].lx, c->mem[mi].ly, 0, nullptr, c->mem[mi].sh, {0, 0, 1}, {}};
    const int start = (int)order.size();
    for (int32_t mj = mi; mj < nmemb; ++mj)
      if (c->mem[mj].lx == k.lx && c->mem[mj].ly == k.ly) order.push_back(mj);
    k.count = (int)order.size() - start;
    k.d_idx = d_idx + start;
    c->cls.push_back(k);
  }
  // Argument tables.
  c->h_args.resize((size_t)kNumTables * nmemb);
  for (int t = 0; t < kNumTables; ++t)
    for (int32_t mi = 0; mi < nmemb; ++mi)
      c->h_args[(size_t)t * nmemb + mi] = member_args(c->mem[mi], c->precision, t);
  const bool ok = hipMemcpyAsync(d_idx, order.data(), order.size() * sizeof(int),
                                 hipMemcpyHostToDevice, c->stream) == hipSuccess &&
                  hipMemcpyAsync(c->d_args, c->h_args.data(),
                                 c->h_args.size() * sizeof(MemberArgs), hipMemcpyHostToDevice,
                                 c->stream) == hipSuccess;
  // the index order must outlive the copies, also when one of them failed
  if (hipStreamSynchronize(c->stream) != hipSuccess || !ok) return fail(CCMSAV_EHIP);
  if (c->persistent) {
    const int r = build_persist_plan(c);
    if (r != CCMSAV_OK) return fail(r);
  }
  if (c->graph) {
    if (hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming) != hipSuccess)
      return fail(CCMSAV_EHIP);
  }
  *out = c;
  return CCMSAV_OK;
}

int ccmsav_init(ccmsav_ctx** out, const ccmsav_params* p, const double* phi0, const double* psi0,
                void* workspace, size_t ws_bytes, void* hip_stream) {
  if (!out || !phi0 || !psi0) return CCMSAV_EINVAL;
  return ccmsav_init_batch(out, 1, p, &phi0, &psi0, workspace, ws_bytes, hip_stream);
}

int ccmsav_step(ccmsav_ctx* c, int32_t nsteps) {
  if (!c || nsteps < 0) return CCMSAV_EINVAL;
  int32_t left = nsteps;
  while (left > 0) {
    if (c->graph && c->level >= 3 && c->level % 3 == 0 && left >= 3) {
      const int r = capture_graph(c);
      if (r != CCMSAV_OK) return r;
      const int reps = left / 3;
      HIP_TRY(hipEventRecord(c->ev_in, c->stream));
      HIP_TRY(hipStreamWaitEvent(c->gstream, c->ev_in, 0));
      for (int i = 0; i < reps; ++i) HIP_TRY(hipGraphLaunch(c->gexec, c->gstream));
      HIP_TRY(hipEventRecord(c->ev_out, c->gstream));
      HIP_TRY(hipStreamWaitEvent(c->stream, c->ev_out, 0));
      c->level += 3 * reps;
      left -= 3 * reps;
      continue;
    }
    const int r = enqueue_step_level(c, c->level, c->stream);
    if (r != CCMSAV_OK) return r;
    c->level += 1;
    left -= 1;
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
      if (enqueue_step_level(c, c->level, c->stream, PhaseEvents{ev + (size_t)nev * s}) !=
          CCMSAV_OK)
        rc = CCMSAV_EHIP;
      c->level += 1;
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

int32_t ccmsav_members(const ccmsav_ctx* c) { return c ? (int32_t)c->mem.size() : -1; }

int ccmsav_energy_m(ccmsav_ctx* c, int32_t member, double* E_mod, double* parts) {
  if (!valid_member(c, member) || !E_mod) return CCMSAV_EINVAL;
  if (c->bdf1 || c->classical) return CCMSAV_EUNSUPPORTED;
  if (c->level < 1) return CCMSAV_EINVAL;
  int r = run_diag(c, member, true);
  if (r != CCMSAV_OK) return r;
  double e[10];
  HIP_TRY(hipMemcpyAsync(e, c->mem[member].ds->energy, sizeof(e), hipMemcpyDeviceToHost,
                         c->stream));
  int err = 0;
  r = read_err_member(c, member, &err);
  if (r != CCMSAV_OK) return r;
  *E_mod = e[0];
  if (parts)
    for (int i = 0; i < 9; ++i) parts[i] = e[1 + i];
  if (err & ERR_MOBILITY) return CCMSAV_EDOMAIN;
  return status_from_err(err);
}

int ccmsav_energy(ccmsav_ctx* c, double* E_mod, double* parts) {
  return ccmsav_energy_m(c, 0, E_mod, parts);
}

int ccmsav_mass_m(ccmsav_ctx* c, int32_t member, double* mass_psi, double* mass_phi) {
  if (!valid_member(c, member)) return CCMSAV_EINVAL;
  int r = run_diag(c, member, false);
  if (r != CCMSAV_OK) return r;
  double t[3];
  HIP_TRY(hipMemcpyAsync(t, c->mem[member].ds->totals, sizeof(t), hipMemcpyDeviceToHost,
                         c->stream));
  int err = 0;
  r = read_err_member(c, member, &err);
  if (r != CCMSAV_OK) return r;
  if (mass_psi) *mass_psi = t[1];
  if (mass_phi) *mass_phi = t[2];
  return status_from_err(err);
}

int ccmsav_mass(ccmsav_ctx* c, double* mass_psi, double* mass_phi) {
  return ccmsav_mass_m(c, 0, mass_psi, mass_phi);
}

int ccmsav_physical_energy_m(ccmsav_ctx* c, int32_t member, double out6[6]) {
  if (!valid_member(c, member) || !out6) return CCMSAV_EINVAL;
  const Member& m = c->mem[member];
  const int sn = (int)(c->level % 3);
  const DiagConst d = make_diag(m.p);
  hipLaunchKernelGGL(k_phys_sums, dim3(m.p.ny), dim3(DIAG_THREADS), 0, c->stream, m.phi[sn],
                     m.psi[sn], m.parte, m.p.nx, m.p.ny, d);
  hipLaunchKernelGGL(k_phys_final, dim3(1), dim3(DIAG_THREADS), 0, c->stream, m.parte, m.p.ny,
                     m.ds, d);
  if (hipGetLastError() != hipSuccess) return CCMSAV_EHIP;
  double t[9];
  HIP_TRY(hipMemcpyAsync(t, m.ds->totals, sizeof(t), hipMemcpyDeviceToHost, c->stream));
  int err = 0;
  const int r = read_err_member(c, member, &err);
  if (r != CCMSAV_OK) return r;
  for (int i = 0; i < 6; ++i) out6[i] = t[3 + i];
  return status_from_err(err);
}

int ccmsav_physical_energy(ccmsav_ctx* c, double out6[6]) {
  return ccmsav_physical_energy_m(c, 0, out6);
}

int ccmsav_get_fields_m(ccmsav_ctx* c, int32_t member, double* phi, double* psi) {
  if (!valid_member(c, member)) return CCMSAV_EINVAL;
  const Member& m = c->mem[member];
  const size_t bytes = (size_t)m.p.nx * m.p.ny * sizeof(double);
  const int s = (int)(c->level % 3);
  if (phi) HIP_TRY(hipMemcpyAsync(phi, m.phi[s], bytes, hipMemcpyDefault, c->stream));
  if (psi) HIP_TRY(hipMemcpyAsync(psi, m.psi[s], bytes, hipMemcpyDefault, c->stream));
  int err = 0;
  const int r = read_err_member(c, member, &err);
  if (r != CCMSAV_OK) return r;
  return status_from_err(err);
}

int ccmsav_get_fields(ccmsav_ctx* c, double* phi, double* psi) {
  return ccmsav_get_fields_m(c, 0, phi, psi);
}

int ccmsav_get_savs_m(ccmsav_ctx* c, int32_t member, double out8[8]) {
  if (!valid_member(c, member) || !out8) return CCMSAV_EINVAL;
  double sav[3][4];
  HIP_TRY(hipMemcpyAsync(sav, c->mem[member].ds->sav, sizeof(sav), hipMemcpyDeviceToHost,
                         c->stream));
  int err = 0;
  const int r = read_err_member(c, member, &err);
  const int64_t n = c->level;
  const int sn = (int)(n % 3), sm = n >= 1 ? (int)((n + 2) % 3) : sn;
  for (int i = 0; i < 4; ++i) {
    out8[i] = sav[sn][i];
    out8[4 + i] = sav[sm][i];
  }
  if (r != CCMSAV_OK) return r;
  return status_from_err(err);
}

int ccmsav_get_savs(ccmsav_ctx* c, double out8[8]) { return ccmsav_get_savs_m(c, 0, out8); }

int64_t ccmsav_level(const ccmsav_ctx* c) { return c ? c->level : -1; }

int ccmsav_set_launch_variants(ccmsav_ctx* c, const int32_t* var3) {
  if (!c || !var3) return CCMSAV_EINVAL;
  for (int t = 0; t < kNumTuned; ++t)
    if (var3[t] < -1 || var3[t] >= kNumVariants) return CCMSAV_EINVAL;
  if (is_gemm(c->precision)) return CCMSAV_EUNSUPPORTED;
  // Finish the work enqueued with the old choice, and drop a graph captured
  // with it (the next graph step captures again).
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (c->gstream) HIP_TRY(hipStreamSynchronize(c->gstream));
  if (c->gexec) {
    (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
  }
  for (SizeClass& k : c->cls)
    for (int t = 0; t < kNumTuned; ++t) {
      if (var3[t] >= 0) k.var[t] = var3[t];
      else if (!c->tuned) k.var[t] = 0;
      if (!c->tuned)
        for (int v = 0; v < kNumVariants; ++v) k.tune_ms[t][v] = 0.0f;
    }
  c->tuned = true;
  return CCMSAV_OK;
}

int32_t ccmsav_tuning(const ccmsav_ctx* c, int32_t max_shapes, int32_t* info, double* ms) {
  if (!c || max_shapes < 0 || (max_shapes > 0 && !info)) return CCMSAV_EINVAL;
  if (!c->tuned) return 0;
  const int32_t n = std::min<int32_t>(max_shapes, (int32_t)c->cls.size());
  for (int32_t s = 0; s < n; ++s) {
    const SizeClass& k = c->cls[s];
    info[5 * s + 0] = 1 << k.lx;
    info[5 * s + 1] = 1 << k.ly;
    for (int t = 0; t < kNumTuned; ++t) info[5 * s + 2 + t] = k.var[t];
    if (ms)
      for (int t = 0; t < kNumTuned; ++t)
        for (int v = 0; v < kNumVariants; ++v)
          ms[6 * s + t * kNumVariants + v] = k.tune_ms[t][v];
  }
  return (int32_t)c->cls.size();
}


int ccmsav_elliptic_solve(ccmsav_ctx* c, const double* rhs, double* out_chi, double* out_zeta) {
  if (!c || !rhs || c->mem.size() != 1) return CCMSAV_EINVAL;
  const int r = set_solve_args(c, c->h_args[(size_t)kSolveTable * c->mem.size()], out_chi,
                               out_zeta);
  if (r != CCMSAV_OK) return r;
  launch_solve(c, rhs);
  return hipGetLastError() == hipSuccess ? CCMSAV_OK : CCMSAV_EHIP;
}

int ccmsav_elliptic_solve_bc(ccmsav_ctx* c, int32_t bc, const double* rhs, double* out_chi,
                             double* out_zeta) {
  if (!c || !rhs || c->mem.size() != 1) return CCMSAV_EINVAL;
  if (bc == CCMSAV_BC_NEUMANN) return ccmsav_elliptic_solve(c, rhs, out_chi, out_zeta);
  if (bc == CCMSAV_BC_PERIODIC) return periodic_solve(c, rhs, out_chi, out_zeta);
  if (bc != CCMSAV_BC_DIRICHLET) return CCMSAV_EINVAL;
  if (is_gemm(c->precision)) return CCMSAV_EUNSUPPORTED;
  const Member& m = c->mem[0];
  const int nx = m.p.nx, ny = m.p.ny;
  const size_t cells = (size_t)nx * ny;
  // Work space in the stencil output region (rewritten by every step): the
  // sign-alternated right-hand side and the two eigenvalue tables.
  double* alt = static_cast<double*>(m.rm);
  double* lx_d = alt + cells;
  double* ly_d = lx_d + nx;
  // Dirichlet eigenvalues of -Delta_h, (4/h^2) sin^2(pi (k+1) / (2 n)) for
  // DST index k, at DCT index N - 1 - k: (4/h^2) cos^2(pi k' / (2 n)).
  std::vector<double> lx(nx), ly(ny);
  for (int k = 0; k < nx; ++k) {
    const double cs = std::cos(M_PI * k / (2.0 * nx));
    lx[k] = 4.0 / (m.p.h * m.p.h) * cs * cs;
  }
  for (int k = 0; k < ny; ++k) {
    const double cs = std::cos(M_PI * k / (2.0 * ny));
    ly[k] = 4.0 / (m.p.h * m.p.h) * cs * cs;
  }
  const bool copied =
      hipMemcpyAsync(lx_d, lx.data(), nx * sizeof(double), hipMemcpyHostToDevice, c->stream) ==
          hipSuccess &&
      hipMemcpyAsync(ly_d, ly.data(), ny * sizeof(double), hipMemcpyHostToDevice, c->stream) ==
          hipSuccess;
  // the host tables must outlive the copies, also when one of them failed
  if (hipStreamSynchronize(c->stream) != hipSuccess || !copied) return CCMSAV_EHIP;
  const dim3 grid((nx + SMOOTH_THREADS - 1) / SMOOTH_THREADS, ny);
  hipLaunchKernelGGL(k_alternate_sign, grid, dim3(SMOOTH_THREADS), 0, c->stream, rhs, alt, nx, ny);
  MemberArgs a = c->h_args[(size_t)kSolveTable * c->mem.size()];
  a.lamx = to_global<const double>(lx_d);
  a.lamy = to_global<const double>(ly_d);
  const int r = set_solve_args(c, a, out_chi, out_zeta);
  if (r != CCMSAV_OK) return r;
  launch_solve(c, alt);
  if (out_chi)
    hipLaunchKernelGGL(k_alternate_sign, grid, dim3(SMOOTH_THREADS), 0, c->stream, out_chi,
                       out_chi, nx, ny);
  if (out_zeta)
    hipLaunchKernelGGL(k_alternate_sign, grid, dim3(SMOOTH_THREADS), 0, c->stream, out_zeta,
                       out_zeta, nx, ny);
  return hipGetLastError() == hipSuccess ? CCMSAV_OK : CCMSAV_EHIP;
}

int ccmsav_smooth_ic(ccmsav_ctx* c, double M, double dt, int32_t nsteps, const double* phi_sharp,
                     double* phi_out) {
  if (!c || !phi_sharp || !phi_out || c->mem.size() != 1 || nsteps < 0) return CCMSAV_EINVAL;
  if (!(M > 0.0) || !(dt > 0.0) || !std::isfinite(M) || !std::isfinite(dt)) return CCMSAV_EINVAL;
  if (is_gemm(c->precision)) return CCMSAV_EUNSUPPORTED;
  const Member& m = c->mem[0];
  const int nx = m.p.nx, ny = m.p.ny;
  const size_t cells = (size_t)nx * ny;
  // The stencil output region holds 8 fields of >= 4 bytes per cell: room for
  // the iterate and the right-hand side in FP64. It is rewritten by every step.
  double* cur = static_cast<double*>(m.rm);
  double* rhs = cur + cells;
  HIP_TRY(hipMemcpyAsync(cur, phi_sharp, cells * sizeof(double), hipMemcpyDefault, c->stream));
  // chi = C1 - C2 Delta_h + C3 Delta_h^2 with C1 = 1/dt, C2 = 0, C3 = M eps
  MemberArgs a = c->h_args[(size_t)kSolveTable * c->mem.size()];
  a.k.C1 = 1.0 / dt;
  a.k.C2 = 0.0;
  a.k.C3 = M * m.p.eps;
  a.k.alpha = 1.0 / dt;      // the unused zeta output stays well defined
  a.k.lam = 0.0;
  const int r = set_solve_args(c, a, cur, nullptr);
  if (r != CCMSAV_OK) return r;
  const dim3 grid((nx + SMOOTH_THREADS - 1) / SMOOTH_THREADS, ny);
  for (int32_t s = 0; s < nsteps; ++s) {
    hipLaunchKernelGGL(k_smooth_rhs, grid, dim3(SMOOTH_THREADS), 0, c->stream, cur, rhs, nx, ny,
                       1.0 / dt, M / m.p.eps, 1.0 / (m.p.h * m.p.h));
    launch_solve(c, rhs);
  }
  const int blocks = (int)std::min<size_t>((cells + SMOOTH_THREADS - 1) / SMOOTH_THREADS, 4096);
  hipLaunchKernelGGL(k_clip_unit, dim3(blocks), dim3(SMOOTH_THREADS), 0, c->stream, cur, cells);
  HIP_TRY(hipMemcpyAsync(phi_out, cur, cells * sizeof(double), hipMemcpyDefault, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return hipGetLastError() == hipSuccess ? CCMSAV_OK : CCMSAV_EHIP;
}

int ccmsav_elliptic_solve_noalloc(const ccmsav_params* p, const double* rhs, double* out_chi,
                                  double* out_zeta, void* hip_stream) {
  if (!rhs) return CCMSAV_EINVAL;
  const int pc = check_params(p);
  if (pc != CCMSAV_OK) return pc;
  if (is_gemm(p->precision)) return CCMSAV_EUNSUPPORTED;
  const int lx = log2_exact(p->nx), ly = log2_exact(p->ny);
  if (lx > kNoallocMaxLog || ly > kNoallocMaxLog) return CCMSAV_EUNSUPPORTED;
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (!on_device(rhs, dev) || (out_chi && !on_device(out_chi, dev)) ||
      (out_zeta && !on_device(out_zeta, dev)))
    return CCMSAV_EINVAL;
  int rc = CCMSAV_OK;
  char* base = noalloc_scratch(&rc);
  if (!base) return rc;
  // Scratch layout (kNoallocLayout); every part 256-byte aligned.
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* q = base + off;
    off += align_up(bytes);
    return q;
  };
  Member m{};
  m.p = *p;
  m.lx = lx;
  m.ly = ly;
  m.sh = stencil_shape(p->nx, p->ny);
  m.mid = take(kNoallocField);
  m.outc = take(2 * kNoallocField);
  m.lamx = reinterpret_cast<double*>(take(kNoallocMaxN * sizeof(double)));
  m.lamy = reinterpret_cast<double*>(take(kNoallocMaxN * sizeof(double)));
  m.unit_coef = reinterpret_cast<double*>(take(8 * sizeof(double)));
  MemberArgs* d_args = reinterpret_cast<MemberArgs*>(take(sizeof(MemberArgs)));
  int* d_idx = reinterpret_cast<int*>(take(sizeof(int)));
  MemberArgs a = member_args(m, p->precision, kSolveTable);
  // An output that is not requested goes to the row-transformed right-hand
  // side's region (FP64-sized), which the column solve has read before the
  // row inverse writes.
  a.phi_new = to_global(out_chi ? out_chi : reinterpret_cast<double*>(m.mid));
  a.psi_new = to_global(out_zeta ? out_zeta : reinterpret_cast<double*>(m.mid));
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  hipLaunchKernelGGL(k_noalloc_setup, dim3(1), dim3(256), 0, st, a, to_global(d_args),
                     to_global(d_idx), to_global(m.lamx), to_global(m.lamy),
                     to_global(m.unit_coef), p->nx, p->ny, p->h);
  const int nx = p->nx, ny = p->ny;
  auto run = [&](auto tm) {
    using TM = decltype(tm);
    using LT = typename Launch<TM>::T;
    LT::t_rd[lx - kMinLog](st, ny, rhs, static_cast<TM*>(m.mid), M_F, ny, nullptr);
    LT::t_col_solve[0][ly - kMinLog](st, nx, Batch{d_args, d_idx, nx});
    const int per = ny / row_idct_rows<TM>(nx, 0);
    LT::t_row_idct[0][lx - kMinLog](st, per, Batch{d_args, d_idx, per});
  };
  if (p->precision != CCMSAV_FP64)
    run(0.0f);
  else
    run(0.0);
  return hipGetLastError() == hipSuccess ? CCMSAV_OK : CCMSAV_EHIP;
}

int ccmsav_pcg_config(ccmsav_ctx* c, double tol, int32_t max_iter) {
  if (!c || !c->classical) return c ? CCMSAV_EUNSUPPORTED : CCMSAV_EINVAL;
  if (!(tol > 0.0) || !std::isfinite(tol) || max_iter < 1 || max_iter > 10000)
    return CCMSAV_EINVAL;
  c->pcg_tol = tol;
  c->pcg_max_iter = max_iter;
  return CCMSAV_OK;
}

int ccmsav_pcg_stats(ccmsav_ctx* c, int32_t iters[2], double rel_residual[2]) {
  if (!c || !iters || !rel_residual) return CCMSAV_EINVAL;
  if (!c->classical) return CCMSAV_EUNSUPPORTED;
  PcgScalars sc{};
  HIP_TRY(hipMemcpyAsync(&sc, c->mem[0].cl_sc, sizeof(sc), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (int s = 0; s < 2; ++s) {
    iters[s] = sc.iters[s];
    rel_residual[s] = sc.bnorm2[s] > 0.0 ? std::sqrt(sc.rnorm2[s] / sc.bnorm2[s]) : 0.0;
  }
  return CCMSAV_OK;
}

int ccmsav_set_spin_limit(ccmsav_ctx* c, uint32_t polls) {
  if (!c) return CCMSAV_EINVAL;
  if (!c->persistent) return CCMSAV_EUNSUPPORTED;
  c->spin_limit = polls;
  return CCMSAV_OK;
}

int ccmsav_destroy(ccmsav_ctx* c) {
  if (!c) return CCMSAV_EINVAL;
  (void)hipStreamSynchronize(c->stream);
  if (c->gstream) (void)hipStreamSynchronize(c->gstream);
  free_ctx(c);
  return CCMSAV_OK;
}

const char* ccmsav_strerror(int code) {
  if (code > 0 || code < CCMSAV_EBARRIER) return "unknown status";
  return kStatusText[-code];
}

}  // extern "C"
