"""The CC-MSAV-BDF1 scheme (App. B remark, every step) on the GPU, through
the C ABI: parity with the oracle's BDF1 trajectory, the mixed path against
the FP64 path, graph replay against eager steps, and the API around it."""
import sys

import numpy as np
import pytest

from oracle import ccmsav_ref as R
from parity_util import envelope, oracle_trajectory, rel_linf, tolerances
from workloads import vesicle_member

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2601_10057_amd import ccmsav as C  # noqa: E402


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def gpu_states(member, steps, precision="fp64", bdf1=True, graph=False):
    out = {}
    with C.Context(member.params, member.phi0, member.psi0, precision, graph=graph,
                   bdf1=bdf1) as ctx:
        for k in range(steps + 1):
            if k > 0:
                ctx.step(1)
            phi, psi = ctx.fields()
            s1, s0 = ctx.savs()
            out[k] = (phi, psi, s1, s0)
    return out


@pytest.mark.parametrize("n", [16, 64, 256])
def test_bdf1_steps_match_oracle(n):
    m = vesicle_member(n, 2601)
    steps = 8
    note(f"bdf1 parity n={n} steps={steps}")
    ref = oracle_trajectory(m.phi0, m.psi0, m.params, steps, bdf1=True)
    pert = oracle_trajectory(m.phi0, m.psi0, m.params, steps, perturb_seed=1, bdf1=True)
    tol = tolerances(envelope(ref, pert))
    got = gpu_states(m, steps)
    for k, (phi, psi, s1, s0) in got.items():
        r = ref[k]
        errs = (rel_linf(phi, r[0]), rel_linf(psi, r[1]), rel_linf(s1, r[2]))
        assert max(errs) <= tol[k], (k, errs, tol[k])


def test_bdf1_rectangular_grid_matches_oracle():
    base = vesicle_member(64, 7)
    phi0 = np.ascontiguousarray(np.concatenate([base.phi0, base.phi0[::-1]], axis=1))
    psi0 = np.ascontiguousarray(np.concatenate([base.psi0, base.psi0[::-1]], axis=1))
    m = type(base)("rect", phi0, psi0, dict(base.params, nx=128, ny=64), {})
    steps = 6
    note("bdf1 parity 128 x 64")
    ref = oracle_trajectory(m.phi0, m.psi0, m.params, steps, bdf1=True)
    pert = oracle_trajectory(m.phi0, m.psi0, m.params, steps, perturb_seed=1, bdf1=True)
    tol = tolerances(envelope(ref, pert))
    got = gpu_states(m, steps)
    for k in (1, 3, steps):
        phi, psi, s1, _ = got[k]
        assert max(rel_linf(phi, ref[k][0]), rel_linf(psi, ref[k][1]),
                   rel_linf(s1, ref[k][2])) <= tol[k], k


def test_bdf1_differs_from_bdf2_after_the_first_step():
    m = vesicle_member(64, 31)
    note("bdf1 vs bdf2 n=64")
    a = gpu_states(m, 3, bdf1=True)
    b = gpu_states(m, 3, bdf1=False)
    # the first step is the BDF1 step in both schemes, bit for bit
    for x, y in zip(a[1], b[1]):
        assert np.array_equal(x, y)
    assert rel_linf(a[3][0], b[3][0]) > 1e-9


def test_bdf1_mixed_path_tracks_fp64_and_conserves_mass():
    m = vesicle_member(512, 5)
    steps = 200
    note(f"bdf1 mixed vs fp64 n=512 steps={steps}")
    with C.Context(m.params, m.phi0, m.psi0, "mixed", bdf1=True) as mx, \
            C.Context(m.params, m.phi0, m.psi0, "fp64", bdf1=True) as fx:
        m0 = mx.mass()[0]
        mx.step(steps)
        fx.step(steps)
        pm, qm = mx.fields()
        pf, qf = fx.fields()
        assert rel_linf(pm, pf) <= 1e-6
        assert rel_linf(qm, qf) <= 1e-6
        assert rel_linf(mx.savs()[0], fx.savs()[0]) <= 1e-6
        assert abs(mx.mass()[0] - m0) <= 1e-13 * abs(m0)
        with pytest.raises(C.CcmsavError) as e:
            mx.energy()
        assert e.value.name == "EUNSUPPORTED"


def test_bdf1_graph_replay_equals_eager_steps():
    ms = [vesicle_member(32, 41), vesicle_member(64, 42), vesicle_member(32, 43)]
    steps = 12
    note(f"bdf1 ensemble graph vs eager, {steps} steps")
    args = ([m.params for m in ms], [m.phi0 for m in ms], [m.psi0 for m in ms], "mixed")
    with C.Context.ensemble(*args, graph=True, bdf1=True) as g, \
            C.Context.ensemble(*args, graph=False, bdf1=True) as e:
        for _ in range(3):
            g.step(steps // 3)
            e.step(steps // 3)
            torch.cuda.synchronize()
            for k in range(len(ms)):
                for x, y in zip(g.fields(k), e.fields(k)):
                    assert np.array_equal(x, y)
    # and each member equals its own oracle BDF1 trajectory to the mixed bound
    ref = R.run(ms[1].phi0, ms[1].psi0, ms[1].params, steps, bdf1=True)
    with C.Context(ms[1].params, ms[1].phi0, ms[1].psi0, "mixed", bdf1=True) as c:
        c.step(steps)
        assert rel_linf(c.fields()[0], ref.phi) <= 1e-6
