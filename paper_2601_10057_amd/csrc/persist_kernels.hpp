// One persistent launch per step of an ensemble (FP32 transforms in increment
// form): the six passes of the step (stencil, row DCT, column Gram, 5x5
// solve, column solve, row inverse; App. B, Algorithm 1, with the transforms
// of App. C) run inside one kernel whose workgroups all stay resident, with a
// grid-wide barrier (grid_barrier.hpp) between consecutive passes.
//
// Every pass calls the same body functions as the one-kernel-per-pass path,
// with the same thread count per body invocation and the same arithmetic, so
// the two paths give bit-identical results (the launch variants of the other
// path are bit-identical among themselves). A workgroup has PS_THREADS
// threads; a body written for NT < PS_THREADS threads runs as PS_THREADS / NT
// sub-groups side by side, each on its own virtual block and its own LDS
// slice, passing the body's workgroup barriers in lockstep: the sub-groups
// of a workgroup always run the same body on the same grid shape, and the
// bodies' barrier sequences do not depend on the block (the column solve's
// k_x = 0 row sums, the one block-dependent part, run with UNIFORM_SYNC).
#pragma once

#include "grid_barrier.hpp"
#include "step_kernels.hpp"

namespace ccm {

constexpr int PS_THREADS = 256;
constexpr int PS_MIN_LOG = 6;        // grids from 64 ...
constexpr int PS_MAX_LOG = 9;        // ... to 512 points per direction
constexpr int PS_MAX_CLASSES = 16;
constexpr int PS_PHASES = 6;
// Launch variants of the tuned bodies used here (all variants agree bit for bit).
constexpr int PS_ROW_DCT_V = 1;
constexpr int PS_COL_SOLVE_V = 0;

// One size class of the ensemble: its grid shape and members.
struct PersistClass {
  int lx, ly;          // log2 of the grid size
  int count;           // members
  const int* idx;      // their argument-table entries
  int sblocks;         // stencil virtual blocks per member
};
// The launch's work list: per pass, the first group of each class (a group is
// the virtual blocks one workgroup takes at once).
struct PersistPlan {
  int ncls;
  PersistClass cls[PS_MAX_CLASSES];
  int off[PS_PHASES][PS_MAX_CLASSES + 1];
};

// LDS slices of sub-groups start at multiples of 256 bytes.
constexpr int ps_stride(size_t bytes) { return (int)((bytes + 255) / 256 * 256); }
__host__ __device__ constexpr int ps_max(int a, int b) { return a > b ? a : b; }

// Threads of one body invocation (pass, grid size n along its transform).
template <typename TM> __host__ __device__ constexpr int ps_body_threads(int pass, int n) {
  return pass == 0 ? STENCIL_THREADS
       : pass == 1 ? line_threads(n)
       : pass == 2 ? gram_threads<TM>(n)
       : pass == 3 ? SOLVE_THREADS_SMALL
       : pass == 4 ? line_threads_v<TM>(n, PS_COL_SOLVE_V)
                   : row_idct_threads<TM>(n, 0);
}
// Virtual blocks per member of a pass on an nx x ny grid.
template <typename TM>
inline int ps_blocks_per_member(int pass, int nx, int ny, int sblocks) {
  switch (pass) {
    case 0: return sblocks;
    case 1: return ny / p1_rows_v<TM>(nx, PS_ROW_DCT_V);
    case 2: return nx / 2;
    case 3: return 1;
    case 4: return nx;                      // two groups (chi, zeta) per strip
    default: return ny / row_idct_rows<TM>(nx, 0);
  }
}

// LDS bytes of the sub-groups of one workgroup for each body and size.
template <typename TM, int N> constexpr int ps_lds_of_size() {
  constexpr int GD = PS_THREADS / line_threads(N);
  constexpr int GG = PS_THREADS / gram_threads<TM>(N);
  constexpr int GS = PS_THREADS / line_threads_v<TM>(N, PS_COL_SOLVE_V);
  constexpr int GI = PS_THREADS / row_idct_threads<TM>(N, 0);
  return ps_max(ps_max(GD * ps_stride(sizeof(RowDctLds<TM, N, PS_ROW_DCT_V>)),
                       GG * ps_stride(sizeof(GramLds<TM, N>))),
                ps_max(GS * ps_stride(sizeof(LinesLds<TM, N, N>)),
                       GI * ps_stride(sizeof(RowIdctBandLds<TM, N>))));
}
template <typename TM> constexpr int ps_lds_bytes() {
  return ps_max(ps_max(ps_stride(sizeof(StencilLds)),
                       ps_stride(sizeof(SolveLds<SOLVE_THREADS_SMALL>))),
                ps_max(ps_max(ps_lds_of_size<TM, 64>(), ps_lds_of_size<TM, 128>()),
                       ps_max(ps_lds_of_size<TM, 256>(), ps_lds_of_size<TM, 512>())));
}

// Agent-scope atomics and fences of the grid barrier (vector memory
// operations). The polls are relaxed loads, so that waiting does not
// invalidate the caches that other workgroups are still working from.
struct DevBarrierOps {
  GridBarrier* b;
  __device__ unsigned load_gen_acquire() {
    return __hip_atomic_load(&b->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
  }
  __device__ unsigned load_gen() {
    return __hip_atomic_load(&b->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __device__ unsigned add_count() {
    return __hip_atomic_fetch_add(&b->count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __device__ void reset_count() {
    __hip_atomic_store(&b->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __device__ void bump_gen() {
    __hip_atomic_fetch_add(&b->gen, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __device__ void acquire_fence() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
  __device__ void release_fence() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
  __device__ unsigned load_err() {
    return __hip_atomic_load(&b->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __device__ void set_err() {
    __hip_atomic_store(&b->err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __device__ void pause() { __builtin_amdgcn_s_sleep(2); }
};

// All global writes of the workgroup are done and released to the device; one
// thread arrives and waits; the workgroup then reads what every other
// workgroup wrote before the barrier. Returns false (uniformly) on a timeout
// or an earlier failure; the barrier's error flag then tells the host. Thread
// 0 also publishes the barrier's index in LDS after its wait: a wave that
// leaves the barrier without seeing it has passed the workgroup barriers out
// of step with thread 0 (a body whose barrier count depends on its block),
// and it flags the failure too (error value 2) instead of going on silently.
__device__ __forceinline__ bool ps_grid_sync(GridBarrier* bar, unsigned spin_limit, int index) {
  __shared__ int ok;
  __shared__ int epoch;
  __builtin_amdgcn_s_waitcnt(0);       // this wave's stores have reached the cache
  __syncthreads();
  if (threadIdx.x == 0) {
    DevBarrierOps o{bar};
    o.release_fence();
    ok = grid_barrier_arrive_wait(o, gridDim.x, spin_limit);
    epoch = index;
  }
  __syncthreads();
  if (epoch != index) {
    if ((threadIdx.x & 63) == 0)
      __hip_atomic_store(&bar->err, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return false;
  }
  return ok != 0;
}

// ---- the passes -------------------------------------------------------------

template <typename TM>
__device__ __forceinline__ void ps_stencil(const PersistClass& c, int grp,
                                           const MemberArgs* __restrict__ tab, char* smem) {
  const MemberArgs& m = tab[c.idx[grp / c.sblocks]];
  const RowArgs a{m.phn, m.phm, m.phmm, m.psn, m.psm, m.psmm};
  stencil_body<TM>(a, static_cast<gptr<TM>>(m.rm), m.part1, m.nx, m.ny, m.iters, m.k,
                   grp % c.sblocks, m.mob_e, m.mob_n, *reinterpret_cast<StencilLds*>(smem),
                   (int)threadIdx.x);
}

template <typename TM, int NX>
__device__ __attribute__((noinline)) void ps_row_dct(const PersistClass& c, int grp,
                                           const MemberArgs* __restrict__ tab, char* smem) {
  constexpr int NT = line_threads(NX), G = PS_THREADS / NT;
  using L = RowDctLds<TM, NX, PS_ROW_DCT_V>;
  const int sg = (int)threadIdx.x / NT;
  const int per = (1 << c.ly) / p1_rows_v<TM>(NX, PS_ROW_DCT_V);
  const int vb = grp * G + sg;
  const MemberArgs& m = tab[c.idx[vb / per]];
  row_dct8_body<TM, NX, PS_ROW_DCT_V>(static_cast<gptr<const TM>>(m.rm),
                                      static_cast<gptr<TM>>(m.mid), m.ny, vb % per,
                                      *reinterpret_cast<L*>(smem + sg * ps_stride(sizeof(L))),
                                      (int)threadIdx.x % NT);
}

template <typename TM, int NY>
__device__ __attribute__((noinline)) void ps_gram(const PersistClass& c, int grp,
                                        const MemberArgs* __restrict__ tab, char* smem) {
  constexpr int NT = gram_threads<TM>(NY), G = PS_THREADS / NT;
  using L = GramLds<TM, NY>;
  const int sg = (int)threadIdx.x / NT;
  const int per = (1 << c.lx) / 2;
  const int vb = grp * G + sg;
  const MemberArgs& m = tab[c.idx[vb / per]];
  const OpConst o{m.k.C1, m.k.C2, m.k.C3, m.k.alpha, m.k.lam};
  col_gram_body<TM, NY, true>(static_cast<gptr<const TM>>(m.mid), m.lamx, m.lamy, m.part2, m.nx, o,
                        vb % per, *reinterpret_cast<L*>(smem + sg * ps_stride(sizeof(L))),
                        (int)threadIdx.x % NT, static_cast<gptr<TM>>(m.rm));
}

__device__ __forceinline__ void ps_solve(const PersistClass& c, int grp,
                                         const MemberArgs* __restrict__ tab, char* smem) {
  const MemberArgs& m = tab[c.idx[grp]];
  solve_body<SOLVE_THREADS_SMALL>(m.part1, m.p1_blocks, m.part2, m.p2_rows, m.ds, m.k,
                                  *reinterpret_cast<SolveLds<SOLVE_THREADS_SMALL>*>(smem),
                                  (int)threadIdx.x);
}

template <typename TM, int NY>
__device__ __attribute__((noinline)) void ps_col_solve(const PersistClass& c, int grp,
                                             const MemberArgs* __restrict__ tab, char* smem) {
  constexpr int NT = line_threads_v<TM>(NY, PS_COL_SOLVE_V), G = PS_THREADS / NT;
  using L = LinesLds<TM, NY, NY>;
  const int sg = (int)threadIdx.x / NT;
  const int per = 1 << c.lx;
  const int vb = grp * G + sg;
  const MemberArgs& m = tab[c.idx[vb / per]];
  const OpConst o{m.k.C1, m.k.C2, m.k.C3, m.k.alpha, m.k.lam};
  col_solve_body<TM, NY, NT, true>(static_cast<gptr<const TM>>(m.mid), m.lamx, m.lamy, m.coef,
                             static_cast<gptr<TM>>(m.outc), m.nx, m.chi_base, m.nchi,
                             m.zeta_base, m.nzeta, m.colsum, o, vb % per,
                             *reinterpret_cast<L*>(smem + sg * ps_stride(sizeof(L))),
                             (int)threadIdx.x % NT);
}

template <typename TM, int NX>
__device__ __attribute__((noinline)) void ps_row_idct(const PersistClass& c, int grp,
                                            const MemberArgs* __restrict__ tab, char* smem) {
  constexpr int NT = row_idct_threads<TM>(NX, 0), G = PS_THREADS / NT;
  using L = RowIdctBandLds<TM, NX>;
  const int sg = (int)threadIdx.x / NT;
  const int per = (1 << c.ly) / row_idct_rows<TM>(NX, 0);
  const int vb = grp * G + sg;
  const MemberArgs& m = tab[c.idx[vb / per]];
  row_idct_band_body<TM, NX>(static_cast<gptr<const TM>>(m.outc), m.phi_new, m.psi_new, m.ny,
                             m.phi_base, m.psi_base, m.colsum, vb % per,
                             *reinterpret_cast<L*>(smem + sg * ps_stride(sizeof(L))),
                             (int)threadIdx.x % NT);
}

// The groups of pass P over all classes, spread over the grid (each XCD takes
// a contiguous range of workgroups, hence of groups in every round): class by
// class, the body chosen by the grid size, each with its own loop.
template <typename TM, int P, typename F>
__device__ __forceinline__ void ps_class_loop(const PersistPlan& pl, int k, F&& body) {
  const int g = (int)gridDim.x;
  const int first = pl.off[P][k], last = pl.off[P][k + 1];
  // this workgroup's first group at or after `first` in the order b, b + g, ...
  const int b = xcd_remap((int)blockIdx.x, g);
  int q = b >= first ? b : b + (first - b + g - 1) / g * g;
  for (; q < last; q += g) {
    body(q - first);
    // The next invocation writes the LDS that slower waves may still be
    // reading (the bodies were written for one invocation per workgroup).
    lds_sync();
  }
}

template <typename TM, int P>
__device__ __forceinline__ void ps_pass(const PersistPlan& pl, const MemberArgs* __restrict__ tab,
                                        char* smem) {
  for (int k = 0; k < pl.ncls; ++k) {
    const PersistClass& c = pl.cls[k];
    if constexpr (P == 0) {
      ps_class_loop<TM, P>(pl, k, [&](int grp) { ps_stencil<TM>(c, grp, tab, smem); });
    } else if constexpr (P == 3) {
      ps_class_loop<TM, P>(pl, k, [&](int grp) { ps_solve(c, grp, tab, smem); });
    } else {
      const int lg = (P == 1 || P == 5) ? c.lx : c.ly;   // length of the transformed lines
      switch (lg) {
#define CCM_PS_CASE(LG)                                                                    \
  case LG:                                                                                 \
    ps_class_loop<TM, P>(pl, k, [&](int grp) {                                             \
      if constexpr (P == 1) ps_row_dct<TM, 1 << LG>(c, grp, tab, smem);                    \
      else if constexpr (P == 2) ps_gram<TM, 1 << LG>(c, grp, tab, smem);                  \
      else if constexpr (P == 4) ps_col_solve<TM, 1 << LG>(c, grp, tab, smem);             \
      else ps_row_idct<TM, 1 << LG>(c, grp, tab, smem);                                    \
    });                                                                                    \
    break;
        CCM_PS_CASE(6)
        CCM_PS_CASE(7)
        CCM_PS_CASE(8)
        CCM_PS_CASE(9)
#undef CCM_PS_CASE
        default:
          break;
      }
    }
  }
}

template <typename TM>
__global__ void __launch_bounds__(PS_THREADS, 2)
k_persist_step(const PersistPlan plan, const MemberArgs* __restrict__ tab, GridBarrier* bar,
               unsigned spin_limit) {
  __shared__ __attribute__((aligned(256))) char smem[ps_lds_bytes<TM>()];
  // a failed barrier of an earlier launch leaves the state unusable
  if (__hip_atomic_load(&bar->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  ps_pass<TM, 0>(plan, tab, smem);
  if (!ps_grid_sync(bar, spin_limit, 1)) return;
  ps_pass<TM, 1>(plan, tab, smem);
  if (!ps_grid_sync(bar, spin_limit, 2)) return;
  ps_pass<TM, 2>(plan, tab, smem);
  if (!ps_grid_sync(bar, spin_limit, 3)) return;
  ps_pass<TM, 3>(plan, tab, smem);
  if (!ps_grid_sync(bar, spin_limit, 4)) return;
  ps_pass<TM, 4>(plan, tab, smem);
  if (!ps_grid_sync(bar, spin_limit, 5)) return;
  ps_pass<TM, 5>(plan, tab, smem);
}

}  // namespace ccm
