// Grid-wide barrier of the persistent step launch: every workgroup of the grid
// arrives once per barrier; the last to arrive resets the arrival count and
// advances the generation, which the others wait for.
//
// The waits are bounded: a workgroup that has polled `spin_limit` times
// without seeing the generation change (a grid larger than the chip holds at
// once, or a host-forced limit in a test of this path) sets the shared error
// flag and returns false, and every other waiting workgroup returns false as
// soon as it sees the flag, so the kernel always ends. After a failure the
// state stays as it is (the error flag set): the launch that owns it must be
// abandoned, and later launches return at once.
//
// The logic is a template over the atomic operations, so that the same code
// runs on the GPU (agent-scope atomics, see persist_kernels.hpp) and in the
// CPU emulation of the tests (std::atomic, one thread per workgroup).
#pragma once

#if defined(__HIPCC__)
#define CCM_HD __host__ __device__
#else
#define CCM_HD
#endif

namespace ccm {

// Barrier state in device memory; all zero before the first launch.
struct GridBarrier {
  unsigned count;   // arrivals at the current barrier
  unsigned gen;     // barriers completed (wraps)
  unsigned err;     // a wait timed out
  unsigned pad;
};

// One arrival (by one thread of the workgroup) and the wait for the rest.
// The caller makes its workgroup's writes visible first (a release fence);
// on success the writes of every workgroup before the barrier are visible to
// the caller afterwards. Ops provides: load_gen_acquire, load_gen (relaxed),
// add_count (relaxed, returns the old count), reset_count, bump_gen (relaxed),
// acquire_fence, release_fence, load_err, set_err, pause.
template <class Ops>
CCM_HD inline bool grid_barrier_arrive_wait(Ops& o, unsigned nblocks, unsigned spin_limit) {
  // The generation is read before arriving (an acquire load, so that the
  // arrival cannot move ahead of it): the last arrival, which advances it,
  // comes after this arrival, so the change cannot be missed.
  const unsigned g = o.load_gen_acquire();
  if (o.add_count() == nblocks - 1) {
    o.acquire_fence();        // the other arrivals' writes (their release fences)
    o.reset_count();
    o.release_fence();        // ... passed on with the new generation
    o.bump_gen();
    return true;
  }
  // Polls are relaxed loads; one acquire fence once the generation changed.
  for (unsigned n = 0;; ++n) {
    if (o.load_gen() != g) {
      o.acquire_fence();
      return true;
    }
    if (o.load_err()) return false;
    if (n >= spin_limit) {
      o.set_err();
      return false;
    }
    o.pause();
  }
}

}  // namespace ccm
