"""CPU emulation of the persistent launch's grid barrier (csrc/grid_barrier.hpp):
the same template, instantiated with std::atomic_ref operations and the
device's fences, one host thread per workgroup, built with g++ (and once
under ThreadSanitizer, which checks that the barrier orders each round's
plain writes before the other threads' reads; it does not model standalone
fences, so that build carries each fence on the atomic operation next to it).

- Rounds: every thread writes its slot, passes the barrier, checks all slots
  of the round, passes a second barrier; several launches in a row reuse the
  state, which each launch leaves with no pending arrivals.
- Bounded waits: a workgroup that never arrives (a grid larger than the chip
  holds) makes every other one return false with the error flag set, and a
  spin limit of zero (as a host would force it in a test) ends every wait at
  once; later launches see the flag and do not wait at all.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2601_10057_amd", "csrc")

SRC = r"""
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>
#include "grid_barrier.hpp"

using ccm::GridBarrier;

// The device's scheme: relaxed operations ordered by explicit fences.
// ThreadSanitizer does not model standalone fences, so its build (OPS_ON_OPS)
// moves each fence onto the atomic operation next to it: the release fence
// before an arrival onto the arrival, the acquire fence after the wait onto
// the poll that sees the new generation, the last arrival's pair onto its
// arrival and its generation update.
#ifndef OPS_ON_OPS
constexpr auto RLX = std::memory_order_relaxed;
constexpr auto ARRIVE = RLX, POLL = RLX, BUMP = RLX;
#else
constexpr auto RLX = std::memory_order_relaxed;
constexpr auto ARRIVE = std::memory_order_acq_rel, POLL = std::memory_order_acquire,
               BUMP = std::memory_order_release;
#endif
struct HostOps {
  GridBarrier* b;
  unsigned load_gen_acquire() {
    return std::atomic_ref<unsigned>(b->gen).load(std::memory_order_acquire);
  }
  unsigned load_gen() { return std::atomic_ref<unsigned>(b->gen).load(POLL); }
  unsigned add_count() { return std::atomic_ref<unsigned>(b->count).fetch_add(1u, ARRIVE); }
  void reset_count() { std::atomic_ref<unsigned>(b->count).store(0u, RLX); }
  void bump_gen() { std::atomic_ref<unsigned>(b->gen).fetch_add(1u, BUMP); }
#ifndef OPS_ON_OPS
  void acquire_fence() { std::atomic_thread_fence(std::memory_order_acquire); }
  void release_fence() { std::atomic_thread_fence(std::memory_order_release); }
#else
  void acquire_fence() {}
  void release_fence() {}
#endif
  unsigned load_err() { return std::atomic_ref<unsigned>(b->err).load(RLX); }
  void set_err() { std::atomic_ref<unsigned>(b->err).store(1u, RLX); }
  void pause() { std::this_thread::yield(); }
};

// mode 0: rounds over several launches; mode 1: one workgroup never arrives;
// mode 2: spin limit zero. argv[5]: the spin limit of modes 0 and 1.
int main(int argc, char** argv) {
  const int mode = std::atoi(argv[1]);
  const unsigned W = (unsigned)std::atoi(argv[2]);
  const int rounds = std::atoi(argv[3]);
  const int launches = std::atoi(argv[4]);
  GridBarrier bar{0, 0, 0, 0};
  std::vector<long> slot(W, -1);
  std::atomic<int> bad{0}, failed{0};
  for (int l = 0; l < launches; ++l) {
    std::vector<std::thread> th;
    const unsigned grid = mode == 1 ? W + 1 : W;   // mode 1: one workgroup never resident
    const unsigned spin = mode == 2 ? 0u : (unsigned)std::atol(argv[5]);
    for (unsigned w = 0; w < W; ++w) {
      th.emplace_back([&, w] {
        HostOps o{&bar};
        if (o.load_err()) { failed++; return; }       // an earlier launch failed
        for (int r = 0; r < rounds; ++r) {
          const long tag = (long)l * rounds + r;
          slot[w] = tag;
          o.release_fence();
          if (!ccm::grid_barrier_arrive_wait(o, grid, spin)) { failed++; return; }
          for (unsigned v = 0; v < W; ++v)
            if (slot[v] != tag) bad++;
          o.release_fence();
          if (!ccm::grid_barrier_arrive_wait(o, grid, spin)) { failed++; return; }
        }
      });
    }
    for (auto& t : th) t.join();
    std::printf("launch %d count %u gen %u err %u bad %d failed %d\n", l, bar.count, bar.gen,
                bar.err, bad.load(), failed.load());
  }
  return 0;
}
"""


def _build(tmp_path, extra=()):
    src = tmp_path / "barrier_emu.cpp"
    src.write_text(SRC)
    exe = tmp_path / ("barrier_emu" + ("_tsan" if extra else ""))
    subprocess.run(["g++", "-std=c++20", "-O2", "-pthread", *extra, "-I", CSRC, str(src), "-o",
                    str(exe)], check=True)
    return exe


def _run(exe, *args, timeout=120):
    out = subprocess.run([str(exe), *map(str, args)], capture_output=True, text=True,
                         timeout=timeout, check=True)
    rows = []
    for line in out.stdout.splitlines():
        f = line.split()
        rows.append({f[i]: int(f[i + 1]) for i in range(0, len(f), 2)})
    return rows, out.stderr


pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


def test_rounds_are_ordered_and_the_state_returns_to_rest(tmp_path):
    exe = _build(tmp_path)
    rows, _ = _run(exe, 0, 24, 300, 4, 200000000)
    for l, r in enumerate(rows):
        assert r["launch"] == l
        assert r["bad"] == 0 and r["failed"] == 0 and r["err"] == 0
        assert r["count"] == 0                     # no arrival left pending
        assert r["gen"] == 2 * 300 * (l + 1)       # two barriers per round


def test_orderings_hold_under_thread_sanitizer(tmp_path):
    exe = _build(tmp_path, ("-fsanitize=thread", "-g", "-DOPS_ON_OPS"))
    env_ok = True
    try:
        rows, err = _run(exe, 0, 8, 200, 2, 200000000, timeout=300)
    except subprocess.CalledProcessError as e:   # a data race makes TSan exit non-zero
        env_ok = False
        err = e.stderr
    assert env_ok and "WARNING: ThreadSanitizer" not in err, err[-2000:]
    assert all(r["bad"] == 0 and r["count"] == 0 for r in rows)


def test_a_workgroup_that_never_arrives_ends_every_wait(tmp_path):
    exe = _build(tmp_path)
    rows, _ = _run(exe, 1, 16, 5, 2, 20000)
    first, second = rows
    assert first["err"] == 1 and first["failed"] == 16 and first["gen"] == 0
    # the next launch sees the flag and returns without waiting
    assert second["failed"] == 32 and second["gen"] == 0


def test_spin_limit_zero_fails_fast(tmp_path):
    exe = _build(tmp_path)
    rows, _ = _run(exe, 2, 16, 50, 1, 0, timeout=30)
    (r,) = rows
    assert r["err"] == 1 and r["failed"] >= 1 and r["bad"] == 0
