"""One persistent kernel launch per ensemble step (CCMSAV_FLAG_PERSISTENT):
all passes of the step for all members inside one launch, with grid-wide
barriers between the passes (the barrier logic is checked in a CPU emulation,
tests/test_grid_barrier_cpu.py).

- Bit-identical to the default path (one launch per pass and grid shape):
  fields and SAVs of every member of mixed-shape ensembles (64^2, 128^2,
  128 x 64, 64 x 128) over 7 steps (the BDF1 first step, the first BDF2 step,
  each phase of the three-level ring twice), with the BDF1 scheme at every
  step as well, and the 48 x 256^2 + 16 x 512^2 workload over 30 steps, with
  its modified energy and mass.
- The captured graph of persistent launches: every replay, with eager work
  and synchronisation between replays, bit-identical to eager steps.
- Failure path, forced from the host: a spin limit of zero makes the grid
  barriers give up; the next synchronising call reports EBARRIER, every
  kernel has ended (the call returns), and later steps return at once.
"""
import sys

import numpy as np
import pytest

from workloads import make_workload, vesicle_member

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2601_10057_amd import ccmsav as C  # noqa: E402


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def members():
    """Grids of 64 and 128 per direction, eps in {3h, 4h, 5h}, rectangles both ways."""
    ms = [vesicle_member(64, 201, c_out_range=(0.8, 1.25), eps_choices=(3.0,)),
          vesicle_member(128, 202, c_out_range=(0.8, 1.25), eps_choices=(5.0,)),
          vesicle_member(64, 203, c_out_range=(0.8, 1.25), eps_choices=(4.0,))]
    base = vesicle_member(64, 204, c_out_range=(0.8, 1.25), eps_choices=(4.0,))
    wide = (np.ascontiguousarray(np.concatenate([base.phi0, base.phi0[:, ::-1]], axis=1)),
            np.ascontiguousarray(np.concatenate([base.psi0, base.psi0[:, ::-1]], axis=1)))
    ms.append(type(base)("wide", *wide, dict(base.params, nx=128, ny=64), {}))
    ms.append(type(base)("tall", np.ascontiguousarray(wide[0].T), np.ascontiguousarray(wide[1].T),
                         dict(base.params, nx=64, ny=128), {}))
    return ms


def states(ctx, n):
    return [(*ctx.fields(m), *ctx.savs(m)) for m in range(n)]


def assert_same(got, ref, what):
    for i, (a, b) in enumerate(zip(got, ref)):
        for x, y in zip(a, b):
            assert np.array_equal(x, y), (what, i)


@pytest.mark.parametrize("bdf1", [False, True])
def test_persistent_steps_are_bit_identical_to_the_default_path(bdf1):
    ms = members()
    args = ([m.params for m in ms], [m.phi0 for m in ms], [m.psi0 for m in ms], "mixed")
    note(f"persistent vs default, {len(ms)} members, bdf1={bdf1}")
    with C.Context.ensemble(*args, persistent=True, bdf1=bdf1) as p, \
            C.Context.ensemble(*args, bdf1=bdf1) as d:
        for chunk in (1, 1, 5):
            p.step(chunk)
            d.step(chunk)
            assert_same(states(p, len(ms)), states(d, len(ms)), (chunk, p.level))
        for i in range(len(ms)):
            assert p.mass(i) == d.mass(i)


def test_graph_of_persistent_launches_matches_eager_steps():
    ms = members()[:4]
    args = ([m.params for m in ms], [m.phi0 for m in ms], [m.psi0 for m in ms], "mixed")
    note("persistent graph vs persistent eager")
    with C.Context.ensemble(*args, persistent=True, graph=True) as g, \
            C.Context.ensemble(*args, persistent=True) as e:
        for chunk in (3, 3, 3, 6, 4, 2, 9):
            g.step(chunk)
            e.step(chunk)
            assert g.level == e.level
            assert_same(states(g, len(ms)), states(e, len(ms)), (chunk, g.level))
            assert g.energy() == e.energy()


def test_ensemble_workload_persistent_matches_default():
    ms = make_workload("ensemble48x256_16x512")
    args = ([m.params for m in ms], [m.phi0 for m in ms], [m.psi0 for m in ms], "mixed")
    note("48 x 256^2 + 16 x 512^2: persistent vs default, 30 steps")
    with C.Context.ensemble(*args, persistent=True) as p, C.Context.ensemble(*args) as d:
        m0 = [p.mass(i)[0] for i in range(len(ms))]
        p.step(30)
        d.step(30)
        assert_same(states(p, len(ms)), states(d, len(ms)), "workload")
        for i in (0, 11, 47, 48, 63):
            assert p.energy(i) == d.energy(i)
        for i in range(len(ms)):
            assert abs(p.mass(i)[0] - m0[i]) <= 5e-11 * abs(m0[i])


def test_barrier_timeout_is_reported_and_every_kernel_ends():
    ms = members()[:2]
    args = ([m.params for m in ms], [m.phi0 for m in ms], [m.psi0 for m in ms], "mixed")
    note("persistent with spin limit 0")
    with C.Context.ensemble(*args, persistent=True) as p:
        p.step(2)
        p.sync()
        p.set_spin_limit(0)
        p.step(1)
        with pytest.raises(C.CcmsavError) as e:
            p.sync()
        assert e.value.name == "EBARRIER"
        p.step(2)            # returns at once on the device
        with pytest.raises(C.CcmsavError) as e:
            p.sync()
        assert e.value.name == "EBARRIER"


def test_spin_limit_is_for_persistent_contexts_only():
    m = members()[0]
    with C.Context(m.params, m.phi0, m.psi0, "mixed") as d:
        with pytest.raises(C.CcmsavError) as e:
            d.set_spin_limit(10)
        assert e.value.name == "EUNSUPPORTED"
