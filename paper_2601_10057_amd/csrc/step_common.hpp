// Shared definitions between the host runtime and the step kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccm {

// Partial sums written by the stencil pass, one row per workgroup.
enum P1Sum {
  P1_RS = 0,      // sum (phi*^2 - 1 - beta)^2 / (4 eps)          -> r_S^2 / h^2
  P1_RW,          // sum 6 phi*^2 |grad phi*|^2 + (phi*^3-phi*)^2/eps^2 -> r_W^2 / h^2
  P1_RZ,          // sum (1 + p) f_in + (1 - p) f_out             -> r_Z^2 / h^2
  P1_ES,          // sum S~ e_phi, e_phi = e0 phi^n + e1 phi^{n-1}
  P1_EH,
  P1_EQ,
  P1_EK,
  P1_EP,          // sum P~ e_psi
  P1_DLAG,        // sum over faces (D delta psi)^2 / M_face of the previous step
  P1_MOBNEG,      // number of faces with M_psi(A phi*) <= 0
  P1_XS,          // increment form only: sum S~ phi^n, H phi^n, Q~ phi^n, K~ phi^n
  P1_XH,
  P1_XQ,
  P1_XK,
  P1_XP,          // increment form only: sum P~ psi^n
  P1_MBAR,        // sum M_psi(phi*) over the cells (classical scheme's preconditioner)
  P1_NSUM
};

// Partial sums of the column pass (Parseval inner products with 1/sigma, 1/tau).
enum P2Sum {
  P2_FS = 0, P2_FH, P2_FQ, P2_FK,            // f_lin with S~, H, Q~, K~
  P2_SS, P2_SH, P2_SQ, P2_SK,
  P2_HH, P2_HQ, P2_HK,
  P2_QQ, P2_QK,
  P2_KK,
  P2_PG, P2_PL,                              // P~ with g_lin, L~ (over tau)
  P2_NSUM
};

// Energy / mass reduction partials, one row each.
enum ESum {
  E_LAP1 = 0,     // ||Lap phi^n||^2 / h^2
  E_LAP2,         // ||Lap (2 phi^n - phi^{n-1})||^2 / h^2
  E_G1,           // face sums of (D phi^n)^2
  E_G2,           // (D (2 phi^n - phi^{n-1}))^2
  E_GD,           // (D (phi^n - phi^{n-1}))^2
  E_P1,           // (phi^n)^2
  E_P2,           // (2 phi^n - phi^{n-1})^2
  E_D,            // (D delta psi)^2 / M_face for the last step
  E_MPSI,         // psi^n
  E_MPHI,         // phi^n
  E_NSUM
};

// Intermediate field slots of the forward transforms.
enum Mid { M_F = 0, M_S, M_H, M_Q, M_K, M_G, M_L, M_P, M_NFIELD };

// Sticky error bits in the device scalar block.
enum ErrBits {
  ERR_NONFINITE = 1,
  ERR_NORM = 2,        // a SAV normaliser r^2 <= tiny
  ERR_PIVOT = 4,       // singular 5x5 system
  ERR_MOBILITY = 8,    // a face mobility <= 0 (energy undefined)
  ERR_PCG = 16,        // the classical scheme's PCG did not reach its tolerance
  ERR_BARRIER = 32,    // a grid barrier of the persistent launch timed out
};

// Device-resident scalar state. Everything the time loop needs lives here so
// that a step never waits on the host.
// Workgroups of the 5x5 kernel per grid of 2048^2 cells or more, each
// reducing a slice of the partial rows.
constexpr int SOLVE_SLICES = 16;

struct DevScalars {
  double sav[3][4];      // V, U, W, Z of the three most recent levels (slot = level % 3)
  double coef[8];        // spectral combination: f, S~, H, Q~, K~ (chi); g, L~ (zeta)
  double acc;            // sum_{j>=2} (dt/2) ||d^j||^2, up to the level before current
  double diag[40];       // last step: s (4), norms r_S r_W r_Z, x (5), M (25), b... see runtime
  double energy[12];     // last energy query: E, then parts
  double totals[16];     // last reduction totals
  double cl[2];          // classical scheme: (P~, zeta^{-1} g), (P~, zeta^{-1} L~)
  int err;
  int pad[3];
  // 5x5 kernel over several workgroups (grids of 2048^2 cells or more): the
  // column sums of each slice of the partial rows, and the slices done in the
  // current step
  double slice[SOLVE_SLICES][P1_NSUM + P2_NSUM];
  unsigned slices_done;
  int pad2[3];
};

// Constants of one step, passed by value to the kernels.
struct StepConst {
  double h, inv_h, inv_h2, h2;
  double eps, beta, M_phi, M0;
  double gamma_in, gamma_out, psi_in, psi_out, beta_in, beta_out;
  double lam, theta_t;
  double x0, x1;         // phi* = x0 phi^n + x1 phi^{n-1}
  double a0, a1;         // a^n = a0 phi^n + a1 phi^{n-1}  (already divided by dt)
  double e0, e1;         // e_phi = e0 phi^n + e1 phi^{n-1} (SAV bracket weights)
  double c0, c1;         // s = c0 SAV^n + c1 SAV^{n-1} + h^2 sum F e
  double alpha;          // 3/(2 dt) or 1/dt
  double C1, C2, C3;     // chi spectrum sigma = C1 + C2 L + C3 L^2
  double C1b;            // C1 - alpha (the surface-energy part of C1)
  double cgs, cga, cgb, cgo;
  double half_dt;
  int lag_d;             // accumulate ||d^n||^2 of the previous (BDF2) step
  int slot_n, slot_m, slot_new;   // SAV ring slots of levels n, n-1, n+1
  int periodic;          // wrap-around ghosts (periodic boundaries), else Neumann
  int classical;         // classical MSAV scheme: lambda div(M grad psi*) in g_lin
};

// Pointer into global memory. The kernels read their pointers from tables in
// device memory; typed in the global address space they are accessed with
// global (not flat) loads and stores.
template <typename T> using gptr = __attribute__((address_space(1))) T*;

template <typename T> inline gptr<T> to_global(T* p) { return (gptr<T>)p; }

// The operator spectra of App. C: sigma = C1 + C2 L + C3 L^2 (chi) and
// tau = alpha + lam L (zeta), with L the eigenvalue of -Delta_h.
struct OpConst {
  double C1, C2, C3, alpha, lam;
};

// State pointers of the three levels a step reads.
struct RowArgs {
  gptr<const double> phn;   // phi^n
  gptr<const double> phm;   // phi^{n-1}
  gptr<const double> phmm;  // phi^{n-2} (lagged ||d||^2 only)
  gptr<const double> psn;
  gptr<const double> psm;
  gptr<const double> psmm;
};

// Everything the kernels of one step need about one grid (one member of an
// ensemble), kept in device memory.
// Strip-major intermediates: strip s (columns 2s, 2s + 1) of a field starts
// strip_stride elements after strip s - 1. The pad beyond the 2 ny values of
// a strip keeps consecutive strips off a power-of-two stride: the row passes
// touch one short piece per strip, and at a stride of 2^k bytes those pieces
// crowd into a few HBM channels (measured at N = 4096: the row DCT takes
// 403 us unpadded, 336 us with this pad; pads of 256 or 4384 bytes are worse).
constexpr int kStripPadBytes = 1056;
__host__ __device__ constexpr size_t strip_stride(int ny, int esize) {
  return 2 * (size_t)ny + (size_t)(kStripPadBytes / esize);
}
// Elements of one strip-major field of an nx x ny grid.
__host__ __device__ constexpr size_t strip_field(int nx, int ny, int esize) {
  return (size_t)(nx / 2) * strip_stride(ny, esize);
}

// FP32 intermediates store the fields in pairs: the two fields of a pair share
// one region, interleaved per row (row j of strip s holds f(2s, j), f(2s+1, j),
// f'(2s, j), f'(2s+1, j): 16 bytes). The row pass then writes a band of rows of
// both fields as one piece (64 bytes for four rows), and the column passes
// load a row of both fields with one 16-byte load. The pairs follow the order
// in which the Gram pass transforms the fields: (S~, H), (Q~, K~), (f_lin, P~),
// (g_lin, L~); the column solve's chi group is f_lin (alone), S~, H, Q~, K~
// and its zeta group g_lin, L~. FP64 intermediates keep one field per region.
// A pair region has the size of one FP64 field region.
__host__ __device__ constexpr int mid_pair(int f) {
  return (f == M_F || f == M_P) ? 0 : (f + 1) / 2;
}
__host__ __device__ constexpr int mid_half(int f) {
  return f == M_P ? 1 : (f == M_F ? 0 : (f + 1) % 2);
}
// Elements (FP32) of one pair strip and of one pair region.
__host__ __device__ constexpr size_t pair_strip_stride(int ny) {
  return 4 * (size_t)ny + (size_t)(kStripPadBytes / 4);
}
__host__ __device__ constexpr size_t pair_field(int nx, int ny) {
  return (size_t)(nx / 2) * pair_strip_stride(ny);
}
static_assert(pair_strip_stride(64) * 4 == strip_stride(64, 8) * 8,
              "a pair region of FP32 fields is the size of one FP64 field region");

struct MemberArgs {
  gptr<const double> phn;        // phi^n, phi^{n-1}, phi^{n-2}
  gptr<const double> phm;
  gptr<const double> phmm;
  gptr<const double> psn;        // psi^n, psi^{n-1}, psi^{n-2}
  gptr<const double> psm;
  gptr<const double> psmm;
  gptr<double> phi_new;          // level n+1 (or the outputs of a standalone solve)
  gptr<double> psi_new;
  gptr<const double> phi_base;   // increment form: phi^n, psi^n added to the increments
  gptr<const double> psi_base;
  gptr<void> rm;                 // 8 stencil fields, row-major
  gptr<void> mid;                // 8 x-transformed fields, strip-major
  gptr<void> outc;               // 2 y-solved fields, strip-major
  gptr<double> part1;            // stencil partial sums, one row per workgroup
  gptr<double> part2;            // column partial sums, one row per strip
  gptr<const double> lamx;       // (4/h^2) sin^2(pi k / (2 n)) per direction
  gptr<const double> lamy;
  gptr<double> colsum;           // increment form: row-sum targets of the psi increment
  gptr<DevScalars> ds;
  gptr<const double> coef;       // spectral combination (ds->coef, or unit weights)
  gptr<double> mob_e;            // classical scheme: M_psi at the east and north face
  gptr<double> mob_n;            //   of each cell (0 on the walls), written by the stencil
  gptr<const int> skip;          // solve kernels return at once while *skip != 0
  int nx, ny;
  int iters, p1_blocks;          // stencil launch shape
  int p2_rows;                   // rows of column partial sums
  int chi_base, nchi, zeta_base, nzeta;   // field groups combined by the column solve
  StepConst k;
};

}  // namespace ccm
