/*
 * ccmsav.h - C ABI of the CC-MSAV vesicle time step on MI355X (gfx950).
 *
 * Zhang, Li, Lowengrub & Wise, "An Efficient Constant-Coefficient MSAV Scheme
 * for Computing Vesicle Growth and Shrinkage", arXiv 2601.10057.
 *
 * The library advances the coupled Allen-Cahn / variable-mobility
 * Cahn-Hilliard vesicle model (Sec. 2.1) in its MSAV form (Sec. 2.2) with the
 * constant-coefficient BDF2 scheme of Sec. 3.2, eqs. (AC_BDF2)-(Z_BDF2), on a
 * cell-centred grid with homogeneous Neumann boundaries (Sec. 3.4, App. D).
 * Each step is solved by the decoupled procedure of App. B (the 5x5 reduced
 * system) with the DCT fast direct solver of App. C; the very first step uses
 * the BDF1 variant of the App. B remark, since BDF2 needs two levels.
 *
 * Conventions for every entry point:
 *  - Scalars are double. Fields are row-major [ny][nx] arrays of double, x
 *    fastest, one value per cell centre ((i + 1/2) h, (j + 1/2) h), no ghosts.
 *  - A field pointer may be host or device memory (copies use
 *    hipMemcpyDefault). The library copies inputs; the caller keeps ownership.
 *  - Every function returns a status (ccmsav_status). On CCMSAV_EINVAL or
 *    CCMSAV_EUNSUPPORTED nothing was changed. Errors detected on the device
 *    are sticky and reported by the next call that synchronises (energy,
 *    mass, get_fields, get_savs, sync). No C++ exception crosses the ABI.
 *  - A context is bound to the stream given at init; all device work of the
 *    context is ordered on that stream. Calls on one context are not
 *    thread-safe.
 */
#ifndef CCMSAV_H
#define CCMSAV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ccmsav_ctx ccmsav_ctx; /* opaque, owned by the library */

typedef enum {
  CCMSAV_OK = 0,
  CCMSAV_EINVAL = -1,       /* invalid argument or parameter */
  CCMSAV_ENOMEM = -2,       /* workspace too small or allocation failed */
  CCMSAV_EHIP = -3,         /* a HIP runtime call failed */
  CCMSAV_EDOMAIN = -4,      /* SAV normaliser <= 0, singular 5x5 system, or a
                               face mobility M_psi <= 0 (energy undefined) */
  CCMSAV_ENONFINITE = -5,   /* NaN or Inf in the state or the SAVs */
  CCMSAV_EUNSUPPORTED = -6, /* grid size or precision mode not provided */
  CCMSAV_ECONVERGE = -7,    /* an iterative solve (CCMSAV_FLAG_CLASSICAL) did not
                               reach its tolerance within its iterations */
  CCMSAV_EBARRIER = -8      /* a grid-wide barrier of the persistent step launch
                               (CCMSAV_FLAG_PERSISTENT) failed (a wait timed out,
                               or the waves of a workgroup left it out of step):
                               the step was abandoned and the context must be
                               destroyed */
} ccmsav_status;

typedef enum {
  CCMSAV_FP64 = 0,          /* all arithmetic in FP64 */
  CCMSAV_MIXED = 1,         /* FP32 transforms; the step is solved for the
                               increments phi^{n+1} - phi^n, psi^{n+1} - psi^n
                               from residuals formed in FP64 (the chi residual
                               uses the biharmonic Delta_h^2 phi^n), and the
                               mean of the psi increment is fixed in FP64 so
                               that h^2 sum psi is conserved to FP64 rounding.
                               FP64 state, SAVs, inner-product sums and 5x5 */
  CCMSAV_MIXED_GEMM_BF16X3 = 2 /* as CCMSAV_MIXED, with every transform on the
                               matrix cores (the library's bf16 MFMA kernels):
                               both operands split into three bfloat16 parts,
                               six products of parts accumulated in FP32 (the
                               rounding of FP32 products). A direction of fewer
                               than 2048 points is a dense product with the DCT
                               matrix; a longer one takes the factored form
                               N = N1 N2 (FFT means: an N1-point and an
                               N2-point DFT product with a twiddle between
                               them). The matrices live in the workspace.
                               Single-member contexts without
                               CCMSAV_FLAG_GRAPH, grids of at least 64 per
                               direction (else EUNSUPPORTED). */
} ccmsav_precision;

/*
 * Problem parameters (paper notation):
 *  nx, ny       grid cells per direction, each a power of two in [16, 8192]
 *  h            cell size (L_x = nx h, L_y = ny h), > 0
 *  dt           time step, > 0
 *  eps          interface width epsilon, > 0                         (Sec. 2.1)
 *  M_phi, M0    Allen-Cahn mobility > 0; M_psi(phi) = 1 - M0 (phi^2 - 1)^2,
 *               0 <= M0 < 1                                           (Sec. 2.1)
 *  gamma_surf, gamma_bend, gamma_area   surface, bending, arc-length weights >= 0
 *  A            arc-length target of F^area; NaN selects the discrete surface
 *               energy of phi0 (so U^0 = 0)
 *  gamma_in, gamma_out, psi_in, psi_out, beta_in, beta_out
 *               osmotic energies f^in/out = gamma/2 (psi - psi_eq)^2 + beta
 *  theta        Allen-Cahn stabilisation >= 0                         (Sec. 3.2)
 *  lam          Cahn-Hilliard stabilisation lambda >= 0               (Sec. 3.2)
 *  beta         linear SAV splitting constant                         (Sec. 2.2)
 *  precision    a ccmsav_precision value
 *  flags        0 or CCMSAV_FLAG_GRAPH, CCMSAV_FLAG_BDF1, CCMSAV_FLAG_PERIODIC,
 *               CCMSAV_FLAG_CLASSICAL, CCMSAV_FLAG_PERSISTENT
 */
typedef struct {
  int32_t nx, ny;
  double h, dt, eps;
  double M_phi, M0;
  double gamma_surf, gamma_bend, gamma_area, A;
  double gamma_in, gamma_out, psi_in, psi_out, beta_in, beta_out;
  double theta, lam, beta;
  int32_t precision, flags;
} ccmsav_params;

/* flags: capture the steady-state steps (level >= 3) once into a HIP graph of
 * three steps and replay it from then on. The graph runs on a stream of the
 * library's own, ordered after and before the context's stream by events. */
#define CCMSAV_FLAG_GRAPH 1

/* flags: take every step with the first-order CC-MSAV-BDF1 scheme (the BDF1
 * remark of App. B: phi* = phi^n, psi* = psi^n, C1 and zeta with 1/dt, and
 * the SAV brackets of level n only) instead of BDF2 after the first step.
 * ccmsav_energy then returns EUNSUPPORTED: E^{n,n-1}_mod is the energy of
 * the BDF2 scheme. */
#define CCMSAV_FLAG_BDF1 2

/* flags: periodic boundaries instead of homogeneous Neumann ones, the case
 * App. C pairs with the FFT. Every discrete operator of App. D takes
 * wrap-around ghosts (the neighbour across a boundary is the cell on the
 * other side of the grid, and the faces across the wrap are faces of the
 * grid), in the step, the initial SAVs and the energy, mass and physical
 * energy queries. Each step is Algorithm 1 of App. B: the seven elliptic
 * solves by the periodic fast solver (the FFT of ccmsav_elliptic_solve_bc
 * with CCMSAV_BC_PERIODIC), the inner products of the 5x5 system in physical
 * space. CCMSAV_FP64 only, single-member contexts without CCMSAV_FLAG_GRAPH,
 * grids up to 4096 per direction (else EUNSUPPORTED). ccmsav_elliptic_solve
 * keeps solving with Neumann boundaries. */
#define CCMSAV_FLAG_PERIODIC 4

/* flags: the classical MSAV scheme of the App. B remarks instead of CC-MSAV,
 * the comparison system of Sec. 4. The Cahn-Hilliard stabilisation sits in the
 * chemical potential: g_lin carries -lambda div(M_psi(phi*) grad psi*) and the
 * operator is zeta = alpha - lambda div(M_psi(phi*) grad), variable in space.
 * Its two solves per step (zeta^{-1} g and zeta^{-1} L~) run as one lock-step
 * conjugate gradient iteration preconditioned with alpha - lambda M_bar
 * Delta_h (M_bar the mean of M_psi(phi*) over the cells, inverted by the DCT
 * solver of App. C), from x = 0 until |r| <= tol |b| (discrete L2 norms),
 * with the mean of x then set from the exact relation alpha sum x = sum b so
 * that mass is conserved to rounding; the Allen-Cahn part and the 5x5
 * reduction are those of CC-MSAV. CCMSAV_FP64 only, single-member contexts
 * with Neumann boundaries, without CCMSAV_FLAG_GRAPH (else EUNSUPPORTED).
 * Not converging within the allowed iterations is a sticky device error
 * (ECONVERGE). ccmsav_energy returns EUNSUPPORTED (E^{n,n-1}_mod with the
 * lambda dissipation sum is the CC-MSAV energy). */
#define CCMSAV_FLAG_CLASSICAL 8

/* flags: every step of the context (Algorithm 1 of App. B with the
 * transforms of App. C, for all members) as ONE persistent kernel launch:
 * the stencil, row DCT, column Gram, 5x5, column solve and row inverse passes
 * run one after the other inside it, separated by grid-wide barriers, on a
 * grid of as many workgroups as the GPU holds at once. The passes are the
 * same computations with the same thread counts as the default launches,
 * and give bit-identical results. A barrier wait that exceeds its spin limit
 * (ccmsav_set_spin_limit; a grid that is not all resident, e.g. beside other
 * work on the GPU) ends every workgroup and is reported as EBARRIER.
 * CCMSAV_MIXED only, Neumann boundaries, the CC-MSAV scheme, grids of 64 to
 * 512 per direction (else EUNSUPPORTED); combines with CCMSAV_FLAG_GRAPH
 * (a graph of three launches) and CCMSAV_FLAG_BDF1. ccmsav_profile_steps
 * reports the whole step as its first phase. */
#define CCMSAV_FLAG_PERSISTENT 16

/* Device workspace bytes a context needs for these parameters (0 if the
 * parameters are invalid or unsupported). */
size_t ccmsav_workspace_bytes(const ccmsav_params* p);

/* Workspace bytes of an ensemble context of nmemb members (0 if invalid). */
size_t ccmsav_workspace_bytes_batch(int32_t nmemb, const ccmsav_params* p);

/*
 * Create a context at level n = 0 from phi0, psi0 (nx*ny doubles each, host or
 * device) and compute the initial SAVs V^0, U^0, W^0, Z^0 (eq. msav_ic).
 * workspace: caller-owned device memory of ws_bytes >= ccmsav_workspace_bytes(p)
 *            that must outlive the context, or NULL to let the library allocate
 *            (and free at destroy).
 * hip_stream: a hipStream_t (NULL = default stream).
 * Returns EINVAL (bad pointer or parameter), EUNSUPPORTED (size / precision),
 * ENOMEM, EHIP, or a device status of the initial reduction (ENONFINITE,
 * EDOMAIN when a SAV normaliser vanishes).
 */
int ccmsav_init(ccmsav_ctx** out, const ccmsav_params* p, const double* phi0, const double* psi0,
                void* workspace, size_t ws_bytes, void* hip_stream);

/*
 * Create a context that advances nmemb >= 1 independent vesicles (an
 * ensemble) in lock step. Member m has its own parameters p[m] and initial
 * fields phi0[m], psi0[m] (p[m].nx * p[m].ny doubles each, host or device);
 * members may differ in grid size, eps, osmotic and all other parameters,
 * but share the precision and the flags. Each kernel of a step is one launch
 * per grid shape covering all members of that shape. Every other entry point
 * applies to all members (step, sync, destroy) or to member 0 (energy, mass,
 * get_fields, get_savs); the _m variants below take a member index.
 * Returns like ccmsav_init; EINVAL also for nmemb outside [1, 4096] or mixed
 * precisions or flags.
 */
int ccmsav_init_batch(ccmsav_ctx** out, int32_t nmemb, const ccmsav_params* p,
                      const double* const* phi0, const double* const* psi0, void* workspace,
                      size_t ws_bytes, void* hip_stream);

/* Number of members of a context (-1 for NULL). */
int32_t ccmsav_members(const ccmsav_ctx* c);

/* Per-member forms of ccmsav_energy, ccmsav_mass, ccmsav_get_fields and
 * ccmsav_get_savs (member in [0, ccmsav_members(c)), else EINVAL). */
int ccmsav_energy_m(ccmsav_ctx* c, int32_t member, double* E_mod, double* parts);
int ccmsav_mass_m(ccmsav_ctx* c, int32_t member, double* mass_psi, double* mass_phi);
int ccmsav_get_fields_m(ccmsav_ctx* c, int32_t member, double* phi, double* psi);
int ccmsav_get_savs_m(ccmsav_ctx* c, int32_t member, double out8[8]);

/*
 * Enqueue nsteps >= 0 time steps (Algorithm 1 of App. B per step; BDF1 for the
 * step from level 0, and for every step under CCMSAV_FLAG_BDF1). Asynchronous:
 * returns once the work is on the stream.
 */
int ccmsav_step(ccmsav_ctx* c, int32_t nsteps);

/*
 * Modified discrete energy E^{n,n-1}_mod of eq. (modified_discrete_energy) at
 * the current level n >= 1, with discrete norms of App. D and the accumulated
 * -sum_{j=2}^{n} (dt/2) ||d^j||^2 (Sec. 3.3). parts (nullable) receives 9
 * values: bending, surface+theta, -theta_tilde term, beta term, V, U, W, Z
 * terms, and minus the accumulated sum. Synchronises the stream.
 * EINVAL if n == 0; EUNSUPPORTED for a context of the BDF1 scheme.
 */
int ccmsav_energy(ccmsav_ctx* c, double* E_mod, double* parts);

/* h^2 sum psi^n (conserved, App. D) and h^2 sum phi^n. Either pointer may be
 * NULL. Synchronises the stream. */
int ccmsav_mass(ccmsav_ctx* c, double* mass_psi, double* mass_phi);

/*
 * Physical free energy of Sec. 2.1 at level n (eq. energy_functional with the
 * densities of eq. energy_densities, in the scheme's discrete forms: cell
 * |grad phi|^2, five-point Delta_h with Neumann ghosts, h^2 sums), into
 * out6 = {F, F^surf, F^bend, F^area, F^osm, int f_surf}; the last is the arc
 * length that F^area holds at A. Synchronises the stream.
 */
int ccmsav_physical_energy(ccmsav_ctx* c, double out6[6]);
int ccmsav_physical_energy_m(ccmsav_ctx* c, int32_t member, double out6[6]);

/* Copy phi^n and psi^n (nx*ny doubles each, host or device; either may be
 * NULL). Synchronises the stream. */
int ccmsav_get_fields(ccmsav_ctx* c, double* phi, double* psi);

/* out8 = {V, U, W, Z} at level n followed by level n-1 (level 0 repeats n). */
int ccmsav_get_savs(ccmsav_ctx* c, double out8[8]);

/* Current level n (number of steps taken). */
int64_t ccmsav_level(const ccmsav_ctx* c);

/*
 * Launch variants chosen by the library's autotuner. At the first step of a
 * context every variant of three kernels is run and timed with HIP events
 * (all variants give bit-identical results) and the fastest is kept: the row
 * DCT-II (variant 1 halves the band of rows per workgroup and its LDS), the
 * column solve and the row DCT-III (variant 0: four elements per thread,
 * variant 1: one FFT butterfly per thread). For each grid shape s of the
 * context (s < max_shapes) info[5 s .. 5 s + 4] = {nx, ny, row DCT variant,
 * column solve variant, row inverse variant} and, if ms is not NULL,
 * ms[6 s .. 6 s + 5] = the best time in milliseconds of variants 0 and 1 of
 * each of the three kernels. Returns the number of grid shapes, 0 before the
 * first step (or for the DCT-as-GEMM precision), EINVAL for bad arguments.
 */
int32_t ccmsav_tuning(const ccmsav_ctx* c, int32_t max_shapes, int32_t* info, double* ms);

/*
 * Fix the launch variants instead of the autotuner's choice: var3[t] for the
 * row DCT, column solve and row inverse (0 or 1, or -1 to keep the current
 * choice; before the first step the current choice is 0). Applies to every
 * grid shape of the context, skips the autotuning of the first step, and
 * drops a captured graph so that the next graph step captures the new
 * launches. All variants compute bit-identical results. Synchronises the
 * stream. EINVAL for a value outside [-1, 1]; EUNSUPPORTED for the
 * DCT-as-GEMM precision, which has no variants.
 */
int ccmsav_set_launch_variants(ccmsav_ctx* c, const int32_t* var3);

/*
 * Take nsteps >= 1 steps like ccmsav_step, with HIP events recorded on the
 * context's stream around each of the six kernels of a step, then wait and
 * write the mean duration in milliseconds of each kernel launch to
 * ms_per_phase[6]: stencil terms, row DCT-II, column DCT-II + inner products,
 * 5x5 solve, column solve (combine, divide, DCT-III), row DCT-III.
 * Creates and destroys 12 * nsteps events (nsteps <= 100000).
 */
int ccmsav_profile_steps(ccmsav_ctx* c, int32_t nsteps, double* ms_per_phase);

/* Wait for the stream and report sticky device errors. */
int ccmsav_sync(ccmsav_ctx* c);

/*
 * Fast direct solver of App. C on its own (single-member contexts only): out_chi = chi^{-1} rhs and
 * out_zeta = zeta^{-1} rhs with the BDF2 operators of App. B Step 3,
 *   chi  = C1 - C2 Delta_h + C3 Delta_h^2, C1 = 3/(2 dt) + M_phi gamma_surf 3 sqrt2 beta/(4 eps),
 *          C2 = M_phi (gamma_surf 3 sqrt2 eps/4 + theta), C3 = M_phi gamma_bend 3 sqrt2 eps/8,
 *   zeta = 3/(2 dt) - lam Delta_h,
 * for the context's parameters. rhs, out_chi, out_zeta: nx*ny doubles in
 * device memory (NULL outputs are skipped). Uses the context's work buffers
 * (not its state); ordered on the context's stream.
 */
int ccmsav_elliptic_solve(ccmsav_ctx* c, const double* rhs, double* out_chi, double* out_zeta);

/* Boundary conditions of the standalone fast direct solver. */
#define CCMSAV_BC_NEUMANN 0
#define CCMSAV_BC_DIRICHLET 1
#define CCMSAV_BC_PERIODIC 2

/*
 * ccmsav_elliptic_solve with a choice of boundary condition. App. C pairs
 * the DCT with homogeneous Neumann boundaries (CCMSAV_BC_NEUMANN, the same
 * as ccmsav_elliptic_solve) and names the DST for homogeneous Dirichlet ones
 * (CCMSAV_BC_DIRICHLET): Delta_h with ghost cells equal to minus their
 * boundary neighbours, diagonalised by the orthonormal DST-II with
 * eigenvalues -(4/h^2)(sin^2(pi (i+1)/(2 nx)) + sin^2(pi (j+1)/(2 ny))).
 * The Dirichlet solve runs the DCT kernels on the input multiplied by
 * (-1)^(i+j), with the eigenvalues re-indexed, and multiplies the outputs by
 * (-1)^(i+j) (a DST-II is a DCT-II of the sign-alternated input read in
 * reverse order). CCMSAV_BC_PERIODIC, the FFT case: Delta_h with wrap-around,
 * diagonal in the Fourier basis with eigenvalues
 * -(4/h^2)(sin^2(pi i/nx) + sin^2(pi j/ny)); FP64 transforms in any
 * precision (two real rows per complex FFT line, half spectra by conjugate
 * symmetry), grids up to 4096 per direction. Same operators, buffers and
 * ordering as ccmsav_elliptic_solve; EINVAL for another bc, EUNSUPPORTED for
 * the DCT-as-GEMM precision with CCMSAV_BC_DIRICHLET and for periodic grids
 * beyond 4096.
 */
int ccmsav_elliptic_solve_bc(ccmsav_ctx* c, int32_t bc, const double* rhs, double* out_chi,
                             double* out_zeta);

/* Bytes of device memory that ccmsav_elliptic_solve_noalloc holds on each GPU
 * the library runs on (a fixed array, kept until the process ends). */
#define CCMSAV_NOALLOC_SCRATCH_BYTES (27u * 1024u * 1024u)

/*
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, and harnesses that forbid hipMalloc. The
 * solve of ccmsav_elliptic_solve without a context: out_chi = chi^{-1} rhs and
 * out_zeta = zeta^{-1} rhs with the BDF2 operators (the constants listed at
 * ccmsav_elliptic_solve) of the parameters p, homogeneous Neumann boundaries,
 * FP64 transforms (p->precision CCMSAV_FP64) or FP32 transforms
 * (CCMSAV_MIXED). The same kernels as ccmsav_elliptic_solve; results agree
 * with it to rounding (the eigenvalue tables are formed on the device).
 *  - p: the parameters of the grid and operators (checked as at init; p->A,
 *    flags and the osmotic parameters are not used). nx, ny powers of two in
 *    [16, 1024].
 *  - rhs: nx*ny doubles, row-major, in device (or managed) memory of the
 *    current device; out_chi, out_zeta likewise, or NULL to skip. Outputs may
 *    not alias rhs. The caller owns all three.
 *  - hip_stream: a hipStream_t of the current device (NULL = default stream).
 *    The work is enqueued on it and the call returns without waiting.
 *  - Scratch: every call uses the library's CCMSAV_NOALLOC_SCRATCH_BYTES array
 *    on the current device, and keeps no state in it between calls (nothing
 *    has to start at zero). Calls on one GPU that overlap in time (other
 *    streams, other host threads) race on that array: order them, for
 *    example on one stream.
 *  - Allocates nothing: no hipMalloc or hipFree and no host-to-device copy;
 *    the tables and the kernels' argument block are written by a kernel. The
 *    first call on a device looks up the array's device address.
 * Returns EINVAL (NULL rhs, bad parameter, a pointer that is not device memory
 * of the current device), EUNSUPPORTED (a grid beyond 1024 per direction,
 * the DCT-as-GEMM precision), EHIP.
 */
int ccmsav_elliptic_solve_noalloc(const ccmsav_params* p, const double* rhs, double* out_chi,
                                  double* out_zeta, void* hip_stream);

/*
 * Smoothed initial phase field (App. F): from phi_sharp, take nsteps steps of
 * the constant-mobility Cahn-Hilliard relaxation phi_t = M Delta(f'(phi)/eps
 * - eps Delta phi), first order and semi-implicit,
 *   (1/dt + M eps Delta_h^2) phi^{k+1} = phi^k/dt + (M/eps) Delta_h((phi^k)^3 - phi^k),
 * with Neumann boundaries, the biharmonic term solved by the fast direct
 * solver of App. C; then clip to [-1, 1] and write phi_out. App. F takes
 * M = 0.01, dt = 1e-6 and ten steps. The grid, h and eps are the context's
 * (single-member contexts), the transforms its precision (FP64, or FP32 for
 * CCMSAV_MIXED). phi_sharp, phi_out: nx*ny doubles, host or device; they may
 * be the same array. Uses the context's work buffers, not its state.
 * Synchronises the stream. EINVAL for NULL pointers, M or dt not positive,
 * nsteps < 0 or an ensemble; EUNSUPPORTED for the DCT-as-GEMM precision.
 */
int ccmsav_smooth_ic(ccmsav_ctx* c, double M, double dt, int32_t nsteps, const double* phi_sharp,
                     double* phi_out);

/*
 * Classical scheme (CCMSAV_FLAG_CLASSICAL): the relative residual tol > 0 at
 * which the conjugate gradient iteration stops (default 1e-12) and the
 * iterations enqueued per step, 1 <= max_iter <= 10000 (default 40; those left
 * after convergence return at once). Applies from the next step.
 * EUNSUPPORTED for a context of another scheme, EINVAL for bad values.
 */
int ccmsav_pcg_config(ccmsav_ctx* c, double tol, int32_t max_iter);

/*
 * Classical scheme: the iterations the last step took for its two solves
 * (iters[0] zeta^{-1} g, iters[1] zeta^{-1} L~) and their final relative
 * residuals |r| / |b|. Synchronises the stream. EUNSUPPORTED for a context of
 * another scheme.
 */
int ccmsav_pcg_stats(ccmsav_ctx* c, int32_t iters[2], double rel_residual[2]);

/*
 * Persistent launch (CCMSAV_FLAG_PERSISTENT): the number of polls (each
 * about a hundred cycles) a workgroup waits at a grid barrier before giving
 * up; 0 gives up at once unless the workgroup arrives last (a way to test
 * the failure path: every kernel still ends normally). Default 1 << 22.
 * Applies from the next step. EUNSUPPORTED for another context.
 */
int ccmsav_set_spin_limit(ccmsav_ctx* c, uint32_t polls);

/* Release the context (and the workspace if the library allocated it). */
int ccmsav_destroy(ccmsav_ctx* c);

/* Static description of a status code. */
const char* ccmsav_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* CCMSAV_H */
