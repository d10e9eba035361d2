"""Mixed-precision step against the FP64 step, both on the GPU.

The mixed path keeps the state, the SAVs, every inner-product sum and the
5x5 system in FP64 and runs the transforms in FP32. On the vesicle family at
N = 2048 and 4096 over 500 steps its phi, psi and U must stay within 1e-6
(relative L-inf) of the FP64 path, its psi mass must drift by at most 5e-11,
and its modified energy must keep decaying.
"""
import sys

import numpy as np
import pytest

from parity_util import rel_linf
from workloads import make_workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2601_10057_amd import ccmsav as C  # noqa: E402

REL_TOL = 1e-6
MASS_DRIFT_TOL = 5e-11


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def run(member, precision, steps, every):
    """States, SAVs, energies and masses every ``every`` steps."""
    out = []
    with C.Context(member.params, member.phi0, member.psi0, precision) as ctx:
        m0 = ctx.mass()[0]
        for k in range(every, steps + 1, every):
            ctx.step(every)
            phi, psi = ctx.fields()
            out.append((k, phi, psi, ctx.savs()[0], ctx.energy(), ctx.mass()[0]))
    return m0, out


@pytest.mark.parametrize("n", [2048, 4096])
def test_mixed_matches_fp64_over_500_steps(n):
    m = make_workload(f"vesicle{n}")[0]
    steps = 500
    note(f"mixed vs fp64 vesicle{n} {steps} steps")
    m0_ref, ref = run(m, "fp64", steps, 100)
    m0_mix, mix = run(m, "mixed", steps, 100)
    assert m0_mix == m0_ref
    worst = {"phi": 0.0, "psi": 0.0, "sav": 0.0, "E": 0.0, "drift": 0.0}
    prev_e = None
    for (k, phi_r, psi_r, s_r, e_r, _), (k2, phi, psi, s, e, mass) in zip(ref, mix):
        assert k == k2
        worst["phi"] = max(worst["phi"], rel_linf(phi, phi_r))
        worst["psi"] = max(worst["psi"], rel_linf(psi, psi_r))
        worst["sav"] = max(worst["sav"], float(np.max(np.abs(s - s_r)) / np.max(np.abs(s_r))))
        worst["E"] = max(worst["E"], abs(e - e_r) / abs(e_r))
        worst["drift"] = max(worst["drift"], abs(mass - m0_mix) / abs(m0_mix))
        if prev_e is not None:
            assert e <= prev_e + 1e-12 * abs(prev_e), (k, e, prev_e)
        prev_e = e
    note("worst " + " ".join(f"{k}={v:.3e}" for k, v in worst.items()))
    assert worst["phi"] <= REL_TOL
    assert worst["psi"] <= REL_TOL
    assert worst["sav"] <= REL_TOL
    assert worst["drift"] <= MASS_DRIFT_TOL
    assert np.isfinite(prev_e)


@pytest.mark.parametrize("n,steps", [(16, 30), (64, 20), (256, 12)])
def test_mixed_matches_oracle_small_grids(n, steps):
    """Against the FP64 oracle directly, on grids the oracle runs in seconds.

    On these coarse grids (eps = 4h is large) the dynamics can amplify small
    perturbations by orders of magnitude within tens of steps, so the bound at
    step k is max(1e-6, 10 x the oracle's own spread under an FP32-sized
    (2^-24 relative) perturbation of the initial fields). At N = 64 the
    FP32 spectra start to be amplified past 1e-6 after about 25 steps (a CPU
    emulation of the same FP32 pipeline shows the same growth), so the
    coarse grids are compared over the first 20-30 steps; the 500-step bound
    is tested above at the benchmark sizes."""
    from oracle import ccmsav_ref as R
    m = make_workload("vesicle1024", n)[0]
    note(f"mixed vs oracle vesicle{n} {steps} steps")
    st = R.initial_state(m.phi0, m.psi0, m.params)
    rng = np.random.default_rng(5)
    u = 2.0 ** -24
    pt = R.initial_state(m.phi0 * (1 + u * rng.choice([-1.0, 1.0], m.phi0.shape)),
                         m.psi0 * (1 + u * rng.choice([-1.0, 1.0], m.psi0.shape)), m.params)
    m0 = R.mass(st)[0]
    worst = 0.0
    with C.Context(m.params, m.phi0, m.psi0, "mixed") as ctx:
        for k in range(steps):
            R.step(st)
            R.step(pt)
            ctx.step(1)
            env = max(rel_linf(pt.phi, st.phi), rel_linf(pt.psi, st.psi))
            tol = max(REL_TOL, 10.0 * env)
            phi, psi = ctx.fields()
            err = max(rel_linf(phi, st.phi), rel_linf(psi, st.psi))
            worst = max(worst, err / tol)
            assert err <= tol, (k, err, env)
            s1, _ = ctx.savs()
            assert np.max(np.abs(s1 - st.sav)) <= tol * np.max(np.abs(st.sav)), k
            assert abs(ctx.mass()[0] - m0) <= MASS_DRIFT_TOL * abs(m0), k
    note(f"worst error / bound = {worst:.3f}")
