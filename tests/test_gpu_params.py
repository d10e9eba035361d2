"""GPU parity off the App. G parameter set, through the C ABI.

Every case here runs general_member's inputs, whose parameters differ from
App. G in every coefficient (M_phi != 1, beta > 0, beta_in != beta_out,
gamma_in != gamma_out, M0, theta, lambda; tests/test_general_params_cpu.py
shows that each slip of those terms moves eight steps by more than 1e-8).
Bars:
- FP64 path against the oracle: max(1e-12, 10 x the oracle's one-ulp
  envelope) on phi, psi and the SAVs (the envelope is near 1e-14, so the bar
  is 1e-12);
- mixed path against the FP64 path: rel L-inf <= 1e-6, mass drift <= 5e-11;
- the modified energy of eq. (modified_discrete_energy) and each of its nine
  parts, evaluated by the library on its own fields, against the oracle's
  formula on the same fields, at 1e-12 of each part's scale (the sum of the
  magnitudes that enter it), over 60 steps so that the accumulated
  dissipation sum is exercised and the beta part is non-zero.
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

MIXED_TOL = 1e-6
MASS_DRIFT = 5e-11
PART_NAMES = ("bend", "surf", "stab", "lin", "V", "U", "W", "Z", "acc")


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def gpu_run(members, steps, precision="fp64", bdf1=False):
    """Fields and SAVs of every member after each step: out[m][k] = (phi, psi, sav, sav_prev)."""
    out = [dict() for _ in members]
    ctx = C.Context.ensemble([m.params for m in members], [m.phi0 for m in members],
                             [m.psi0 for m in members], precision, bdf1=bdf1)
    with ctx:
        for k in range(steps + 1):
            if k > 0:
                ctx.step(1)
            for i in range(len(members)):
                phi, psi = ctx.fields(i)
                s1, s0 = ctx.savs(i)
                out[i][k] = (phi, psi, s1, s0)
    return out


def check_against_oracle(member, got, steps, bdf1=False):
    ref = oracle_trajectory(member.phi0, member.psi0, member.params, steps, bdf1=bdf1)
    pert = oracle_trajectory(member.phi0, member.psi0, member.params, steps, perturb_seed=1,
                             bdf1=bdf1)
    tol = tolerances(envelope(ref, pert))
    worst = 0.0
    for k in range(steps + 1):
        phi, psi, s1, s0 = got[k]
        r = ref[k]
        errs = (rel_linf(phi, r[0]), rel_linf(psi, r[1]), rel_linf(s1, r[2]))
        assert max(errs) <= tol[k], (member.name, k, errs, tol[k])
        if k >= 1:
            assert rel_linf(s0, r[3]) <= tol[k - 1], (member.name, k)
        worst = max(worst, max(errs))
    return worst


CASES = [(16, 16, 0, 4.0), (64, 64, 0, 4.0), (256, 256, 0, 4.0), (128, 64, 0, 4.0),
         (32, 64, 3, 4.0), (64, 32, 2, 5.0), (32, 32, 1, 3.0)]


@pytest.mark.parametrize("nx,ny,variant,eps_cells", CASES)
def test_fp64_steps_match_oracle(nx, ny, variant, eps_cells):
    m = general_member(nx, ny, 10057, variant, eps_cells)
    note(f"general fp64 {nx}x{ny} set {variant} eps {eps_cells}h, 8 steps")
    got = gpu_run([m], 8)[0]
    worst = check_against_oracle(m, got, 8)
    note(f"  worst rel err {worst:.2e}")


@pytest.mark.parametrize("nx,ny,variant", [(16, 16, 0), (64, 64, 0), (128, 64, 0),
                                           (32, 64, 3)])
def test_bdf1_scheme_matches_oracle(nx, ny, variant):
    m = general_member(nx, ny, 10057, variant)
    note(f"general bdf1 {nx}x{ny} set {variant}, 8 steps")
    got = gpu_run([m], 8, bdf1=True)[0]
    check_against_oracle(m, got, 8, bdf1=True)


@pytest.mark.parametrize("nx,ny,variant", [(16, 16, 0), (64, 64, 0), (256, 256, 0),
                                           (128, 64, 0), (32, 64, 3)])
def test_mixed_matches_fp64(nx, ny, variant):
    m = general_member(nx, ny, 10057, variant)
    steps = 40
    note(f"general mixed vs fp64 {nx}x{ny} set {variant}, {steps} steps")
    f64 = gpu_run([m], steps, "fp64")[0]
    mix = gpu_run([m], steps, "mixed")[0]
    h2 = m.params["h"] ** 2
    m0 = h2 * f64[0][1].sum()
    worst = 0.0
    for k in range(steps + 1):
        a, b = mix[k], f64[k]
        e = max(rel_linf(a[0], b[0]), rel_linf(a[1], b[1]), rel_linf(a[2], b[2]))
        assert e <= MIXED_TOL, (k, e)
        worst = max(worst, e)
        drift = abs(h2 * a[1].sum() - m0) / abs(m0)
        assert drift <= MASS_DRIFT, (k, drift)
    note(f"  worst rel err {worst:.2e}")


def test_ensemble_with_mixed_parameters_matches_oracle():
    """Members of one context with different parameter sets, grids and eps:
    every member against its own oracle trajectory (FP64), and the mixed
    ensemble against the FP64 one."""
    members = [general_member(32, 32, 11, 1, 3.0), general_member(64, 32, 12, 2, 5.0),
               general_member(32, 64, 13, 3, 4.0), general_member(64, 64, 14, 0, 4.0),
               general_member(32, 32, 15, 2, 4.0)]
    steps = 8
    note(f"general ensemble fp64 {len(members)} members, {steps} steps")
    got = gpu_run(members, steps, "fp64")
    for m, g in zip(members, got):
        check_against_oracle(m, g, steps)
    note("general ensemble mixed vs fp64")
    mix = gpu_run(members, steps, "mixed")
    for g64, gm in zip(got, mix):
        for k in range(steps + 1):
            assert max(rel_linf(gm[k][0], g64[k][0]), rel_linf(gm[k][1], g64[k][1])) <= MIXED_TOL


# ------------------------------------------------------------------ energy

def energy_scales(phi1, phi0, sav1, sav0, d_terms, p):
    """Scale of each part of E_mod: the sum of the magnitudes that enter it.
    All parts are sums of squares with one sign, except the theta~ part
    -tt/2 (g1 + g2 - 2 gd), whose scale is tt/2 (g1 + g2 + 2 gd)."""
    h = p.h
    g1 = R.grad_norm_sq(phi1, h)
    g2 = R.grad_norm_sq(2.0 * phi1 - phi0, h)
    gd = R.grad_norm_sq(phi1 - phi0, h)
    ref = R.modified_energy(phi1, phi0, sav1, sav0, sum(d_terms), p)
    sc = {k: abs(ref[k]) for k in PART_NAMES}
    sc["stab"] = 0.5 * R.theta_tilde(p) * (g1 + g2 + 2.0 * gd)
    sc["acc"] = sum(abs(t) for t in d_terms)
    sc["E"] = sum(sc[k] for k in PART_NAMES)
    return ref, sc


def d_term(levels, j, p):
    """(dt/2) ||d^j||^2 of the step that produced level j from levels j-1, j-2."""
    phi_m2, psi_m2 = levels[j - 2][:2]
    phi_m1, psi_m1 = levels[j - 1][:2]
    psi_j = levels[j][1]
    return 0.5 * p.dt * R.d_norm_sq(psi_j, 2.0 * psi_m1 - psi_m2, 2.0 * phi_m1 - phi_m2, p)


@pytest.mark.parametrize("nx,ny,variant", [(64, 64, 0), (32, 64, 3)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_energy_parts_match_oracle_on_own_fields(nx, ny, variant, precision):
    """E_mod and its nine parts at 1e-12 of their scales after 2 .. 60 steps.

    The oracle evaluates eq. (modified_discrete_energy) on the library's own
    levels n and n-1 and SAVs, with the dissipation sum rebuilt from the
    library's levels (so the comparison is of the diagnostic, not of the
    trajectory, which the other tests bound)."""
    m = general_member(nx, ny, 10057, variant)
    p = R.initial_state(m.phi0, m.psi0, m.params).p
    steps = 60
    note(f"energy parts {nx}x{ny} set {variant} {precision}, {steps} steps")
    levels = {}
    d_terms = []
    with C.Context(m.params, m.phi0, m.psi0, precision) as ctx:
        for k in range(steps + 1):
            if k > 0:
                ctx.step(1)
            phi, psi = ctx.fields()
            s1, s0 = ctx.savs()
            levels[k] = (phi, psi, s1, s0)
            if k >= 2:
                d_terms.append(d_term(levels, k, p))
            if k in (1, 2, 3, 10, 30, 60):
                e, parts = ctx.energy(parts=True)
                ref, sc = energy_scales(phi, levels[k - 1][0], s1, s0, d_terms, p)
                got = dict(zip(PART_NAMES, parts))
                got["E"] = e
                assert abs(ref["lin"]) > 0.0
                if k >= 3:
                    assert abs(ref["acc"]) > 0.0
                for name in PART_NAMES + ("E",):
                    err = abs(got[name] - ref[name])
                    assert err <= 1e-12 * sc[name], (k, name, got[name], ref[name], sc[name])


def test_energy_along_oracle_trajectory():
    """The library's E_mod against the oracle's along the oracle trajectory
    (64^2, 60 steps, FP64): the trajectories agree to the field bar, so E_mod
    and its parts agree to about that bar times the Laplacian's
    amplification of field differences (8/h^2 against 1/eps^2, 128 for
    eps = 4h); the bound is 1e-10 of the part scales, with the measured
    difference printed. Mass is conserved to 1e-13 and E_mod decreases."""
    m = general_member(64, 64, 10057, 0)
    steps = 60
    note(f"energy along trajectory 64x64, {steps} steps")
    st = R.initial_state(m.phi0, m.psi0, m.params)
    p = st.p
    worst = 0.0
    prev = None
    with C.Context(m.params, m.phi0, m.psi0) as ctx:
        m0 = ctx.mass()[0]
        for k in range(1, steps + 1):
            R.step(st)
            ctx.step(1)
            e, parts = ctx.energy(parts=True)
            ref = R.energy(st)
            _, sc = energy_scales(st.phi, st.phi_prev, st.sav, st.sav_prev,
                                  [-ref["acc"]], p)
            got = dict(zip(PART_NAMES, parts))
            got["E"] = e
            for name in PART_NAMES + ("E",):
                err = abs(got[name] - ref[name]) / sc[name] if sc[name] > 0 else 0.0
                worst = max(worst, err)
                assert err <= 1e-10, (k, name, got[name], ref[name])
            assert abs(ctx.mass()[0] - m0) <= 1e-13 * abs(m0)
            if prev is not None:
                assert e <= prev + 1e-12 * abs(prev)
            prev = e
    note(f"  worst scaled energy difference {worst:.2e}")
