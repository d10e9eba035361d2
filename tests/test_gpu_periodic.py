"""The time step with periodic boundaries (CCMSAV_FLAG_PERIODIC) through the C
ABI, against the oracle's periodic step (tests/test_oracle_periodic.py pins
it): wrap-around ghosts in every operator, the seven solves of Algorithm 1
by the FFT solver, the inner products in physical space.

The inputs are general_member's vesicles moved by a cyclic shift so that
they straddle both wrap-around seams, with the general parameter sets (every
coefficient off App. G). Bars: FP64 at max(1e-12, 10 x the oracle's one-ulp
envelope); the initial SAVs, energy parts and physical energy at 1e-12 of
their scales; mass exact to 1e-13; cyclic translations commute with the
step to 1e-12; at N = 1024 the BDF1 and BDF2 steps satisfy the discrete
equations (step residuals, every mode weighed alike) within 1e-12.
"""
import sys

import numpy as np
import pytest

from oracle import ccmsav_ref as R
from parity_util import envelope, oracle_trajectory, rel_linf, tolerances
from workloads import general_member

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2601_10057_amd import ccmsav as C  # noqa: E402

PART_NAMES = ("bend", "surf", "stab", "lin", "V", "U", "W", "Z", "acc")


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


class Shifted:
    """general_member's vesicle moved across both seams, periodic parameters."""

    def __init__(self, nx, ny, variant=0, seed=10057):
        m = general_member(nx, ny, seed, variant)
        sh = (ny // 2 - 3, nx // 2 + 5)
        self.phi0 = np.ascontiguousarray(np.roll(m.phi0, sh, (0, 1)))
        self.psi0 = np.ascontiguousarray(np.roll(m.psi0, sh, (0, 1)))
        self.params = dict(m.params, bc="periodic")
        self.name = f"periodic{nx}x{ny}_v{variant}"


def gpu_levels(m, steps, bdf1=False):
    out = {}
    with C.Context(m.params, m.phi0, m.psi0, "fp64", bdf1=bdf1, periodic=True) as ctx:
        for k in range(steps + 1):
            if k:
                ctx.step(1)
            phi, psi = ctx.fields()
            s1, s0 = ctx.savs()
            out[k] = (phi, psi, s1, s0)
    return out


@pytest.mark.parametrize("nx,ny,variant,bdf1", [(16, 16, 0, False), (64, 64, 0, False),
                                                (256, 256, 0, False), (128, 64, 0, False),
                                                (32, 64, 3, False), (64, 64, 1, True),
                                                (128, 64, 2, True)])
def test_periodic_steps_match_oracle(nx, ny, variant, bdf1):
    m = Shifted(nx, ny, variant)
    steps = 8
    note(f"{m.name} bdf1={bdf1}, {steps} steps")
    ref = oracle_trajectory(m.phi0, m.psi0, m.params, steps, bdf1=bdf1)
    pert = oracle_trajectory(m.phi0, m.psi0, m.params, steps, perturb_seed=1, bdf1=bdf1)
    tol = tolerances(envelope(ref, pert))
    got = gpu_levels(m, steps, bdf1)
    worst = 0.0
    for k in range(steps + 1):
        phi, psi, s1, s0 = got[k]
        errs = (rel_linf(phi, ref[k][0]), rel_linf(psi, ref[k][1]), rel_linf(s1, ref[k][2]))
        assert max(errs) <= tol[k], (k, errs, tol[k])
        worst = max(worst, max(errs))
    note(f"  worst rel err {worst:.2e}")


def test_cyclic_translation_commutes_with_the_step():
    m = Shifted(128, 128)
    sh = (37, 71)
    moved = Shifted(128, 128)
    moved.phi0 = np.ascontiguousarray(np.roll(m.phi0, sh, (0, 1)))
    moved.psi0 = np.ascontiguousarray(np.roll(m.psi0, sh, (0, 1)))
    note("periodic translation 128x128, 6 steps")
    a = gpu_levels(m, 6)[6]
    b = gpu_levels(moved, 6)[6]
    assert rel_linf(b[0], np.roll(a[0], sh, (0, 1))) <= 1e-12
    assert rel_linf(b[1], np.roll(a[1], sh, (0, 1))) <= 1e-12
    assert rel_linf(b[2], a[2]) <= 1e-12


def test_periodic_initial_savs_energy_parts_mass_and_physical_energy():
    m = Shifted(64, 64)
    p = R.initial_state(m.phi0, m.psi0, m.params).p
    steps = 30
    note(f"{m.name} energy parts, {steps} steps")
    levels, d_terms = {}, []
    with C.Context(m.params, m.phi0, m.psi0, "fp64", periodic=True) as ctx:
        s1, _ = ctx.savs()
        ref0 = R.initial_state(m.phi0, m.psi0, m.params)
        assert rel_linf(s1, ref0.sav) <= 1e-12
        m0 = ctx.mass()[0]
        assert m0 == pytest.approx(R.mass(ref0)[0], rel=1e-13)
        ph = ctx.physical_energy()
        ref_ph = R.physical_energy(m.phi0, m.psi0, p)
        for key in ("surf", "bend", "osm", "arc_length"):
            assert ph[key] == pytest.approx(ref_ph[key], rel=1e-12), key
        for k in range(steps + 1):
            if k:
                ctx.step(1)
            phi, psi = ctx.fields()
            s1, s0 = ctx.savs()
            levels[k] = (phi, psi)
            if k >= 2:
                (pm2, qm2), (pm1, qm1) = levels[k - 2], levels[k - 1]
                d_terms.append(0.5 * p.dt * R.d_norm_sq(psi, 2.0 * qm1 - qm2, 2.0 * pm1 - pm2, p))
            if k in (1, 2, 10, 30):
                e, parts = ctx.energy(parts=True)
                ref = R.modified_energy(phi, levels[k - 1][0], s1, s0, sum(d_terms), p)
                g1 = R.grad_norm_sq(phi, p.h, p.bc)
                g2 = R.grad_norm_sq(2.0 * phi - levels[k - 1][0], p.h, p.bc)
                gd = R.grad_norm_sq(phi - levels[k - 1][0], p.h, p.bc)
                sc = {n: abs(ref[n]) for n in PART_NAMES}
                sc["stab"] = 0.5 * R.theta_tilde(p) * (g1 + g2 + 2.0 * gd)
                sc["acc"] = sum(abs(t) for t in d_terms)
                sc["E"] = sum(sc[n] for n in PART_NAMES)
                got = dict(zip(PART_NAMES, parts))
                got["E"] = e
                for n in PART_NAMES + ("E",):
                    assert abs(got[n] - ref[n]) <= 1e-12 * sc[n], (k, n, got[n], ref[n])
            assert abs(ctx.mass()[0] - m0) <= 1e-13 * abs(m0)


def test_periodic_bench_sized_steps_satisfy_the_discrete_equations():
    m = Shifted(1024, 1024)
    note("periodic 1024^2: residuals of the BDF1 and BDF2 steps")
    got = gpu_levels(m, 2)
    p = R.Params.from_dict(m.params)
    lv = [(got[k][0], got[k][1], got[k][2]) for k in range(3)]
    r1 = R.step_residuals(*lv[0], *lv[1], p)
    r2 = R.step_residuals(*lv[1], *lv[2], p, *lv[0])
    note(f"  bdf1 {r1}\n  bdf2 {r2}")
    for r in (r1, r2):
        assert max(r.values()) <= 1e-12, r
