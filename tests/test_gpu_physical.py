"""Physical free energy and arc length (Sec. 2.1) on the GPU through the C
ABI, against the oracle: at the initial level and along trajectories, FP64
and FP32-transform contexts, ensemble members and a rectangular grid."""
import sys

import numpy as np
import pytest

from oracle import ccmsav_ref as R
from workloads import make_workload, vesicle_member

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2601_10057_amd import ccmsav as C  # noqa: E402

KEYS = ("F", "surf", "bend", "area", "osm", "arc_length")


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def resolved(m):
    """Parameters with the arc-length target A resolved as the library does."""
    return R.initial_state(m.phi0, m.psi0, m.params).p


def close(got, ref, p, rtol=1e-12):
    """Each part to rtol of its size; F^area = gamma_area (L - A)^2 / 2 also to
    rtol of its first-order sensitivity gamma_area (|L - A| + 1e-12 L) L to
    the arc length L, since L - A cancels (A itself is a sum of the same
    densities, taken by another reduction)."""
    for k in KEYS:
        scale = abs(ref[k])
        if k in ("area", "F"):
            L = abs(ref["arc_length"])
            scale += p.gamma_area * (abs(ref["arc_length"] - p.A) + 1e-12 * L) * L
        assert abs(got[k] - ref[k]) <= rtol * max(scale, 1e-300), (k, got[k], ref[k])


@pytest.mark.parametrize("n", [64, 256])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_physical_energy_matches_oracle_along_a_trajectory(n, precision):
    m = vesicle_member(n, 21)
    note(f"physical energy n={n} {precision}")
    with C.Context(m.params, m.phi0, m.psi0, precision) as ctx:
        p = resolved(m)
        close(ctx.physical_energy(), R.physical_energy(m.phi0, m.psi0, p), p)
        for _ in range(5):
            ctx.step(1)
            phi, psi = ctx.fields()
            # the GPU's own fields: the diagnostic itself is compared, not the step
            close(ctx.physical_energy(), R.physical_energy(phi, psi, p), p)


def test_physical_energy_of_ensemble_members_and_a_rectangular_grid():
    base = vesicle_member(32, 7)
    phi0 = np.ascontiguousarray(np.concatenate([base.phi0, base.phi0[::-1]], axis=1))
    psi0 = np.ascontiguousarray(np.concatenate([base.psi0, base.psi0[::-1]], axis=1))
    rect = type(base)("rect", phi0, psi0, dict(base.params, nx=64, ny=32), {})
    ms = [vesicle_member(64, 8), rect, vesicle_member(32, 9)]
    note("physical energy ensemble")
    with C.Context.ensemble([m.params for m in ms], [m.phi0 for m in ms],
                            [m.psi0 for m in ms]) as ens:
        ens.step(3)
        for k, m in enumerate(ms):
            phi, psi = ens.fields(k)
            p = resolved(m)
            close(ens.physical_energy(member=k), R.physical_energy(phi, psi, p), p)
        with pytest.raises(C.CcmsavError):
            ens.physical_energy(member=len(ms))


def test_physical_energy_on_the_circle_workload_tracks_the_oracle():
    """circle128 after 20 steps: the GPU's diagnostic of its own state against
    the oracle's diagnostic of the oracle's state (both trajectories agree to
    their rounding envelope, far below this bound)."""
    m = make_workload("circle128")[0]
    note("physical energy circle128, 20 steps")
    st = R.initial_state(m.phi0, m.psi0, m.params)
    for _ in range(20):
        R.step(st)
    ref = R.physical_energy(st.phi, st.psi, st.p)
    with C.Context(m.params, m.phi0, m.psi0) as ctx:
        ctx.step(20)
        close(ctx.physical_energy(), ref, st.p, rtol=1e-9)
