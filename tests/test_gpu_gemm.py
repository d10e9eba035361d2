"""The DCT-as-GEMM variant (products on the matrix cores, FP32 accumulation)
against the FP64 path and the oracle.

Every product splits both operands into three bf16 parts and takes the six
products of parts that carry FP32 accuracy, so the variant rounds like the
mixed path's FP32 transforms. Directions of fewer than 2048 points are dense
products with the DCT matrix; longer ones take the factored form (N1-point
and N2-point DFT products with a twiddle between them). Bounds against the
FP64 path: 1e-6 on the perturbed-vesicle grids (N = 512 dense, 2048
factored; measured 2.0e-7 and 5e-8, the mixed path 1.0e-7 on the first),
whose steps change the fields by a small fraction; 5e-5 on circle128, whose
time step of 1e-4 changes them by up to a few percent per step (measured
2.2e-5 after 100 steps; the mixed path 9e-6). A wrong sign, index or
transpose anywhere in the products gives O(1) errors. Mass stays exact to
FP64 rounding and the modified energy keeps decaying.
"""
import sys

import numpy as np
import pytest

from parity_util import rel_linf
from workloads import make_workload, circle_member, vesicle_member

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2601_10057_amd import ccmsav as C  # noqa: E402


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def run(m, precision, steps, every):
    out = []
    with C.Context(m.params, m.phi0, m.psi0, precision) as ctx:
        m0 = ctx.mass()[0]
        for k in range(every, steps + 1, every):
            ctx.step(every)
            out.append((k, *ctx.fields(), ctx.savs()[0], ctx.energy(), ctx.mass()[0]))
    return m0, out


@pytest.mark.parametrize("name,n,steps,tol", [("circle128", None, 100, 5e-5),
                                              ("vesicle1024", 512, 60, 1e-6),
                                              ("vesicle2048", None, 100, 1e-6)])
def test_gemm_variant_tracks_fp64(name, n, steps, tol):
    m = make_workload(name, n)[0]
    note(f"gemm vs fp64 {name} n={m.params['nx']} {steps} steps")
    m0, ref = run(m, "fp64", steps, steps // 4)
    m0g, got = run(m, "gemm", steps, steps // 4)
    assert m0g == m0
    worst = 0.0
    drift = 0.0
    prev = None
    for r, g in zip(ref, got):
        worst = max(worst, rel_linf(g[1], r[1]), rel_linf(g[2], r[2]))
        drift = max(drift, abs(g[5] - m0) / abs(m0))
        if prev is not None:
            assert g[4] <= prev + 1e-12 * abs(prev)
        prev = g[4]
    note(f"worst rel L-inf {worst:.3e}, mass drift {drift:.2e}")
    assert worst <= tol
    assert drift <= 5e-11


def mirrored_tiles(m, rx, ry):
    """rx x ry copies of a member's fields, every other copy mirrored, so that
    the tiled fields stay smooth and satisfy the Neumann condition at the seams."""
    def tile(f):
        row = np.concatenate([f if i % 2 == 0 else f[:, ::-1] for i in range(rx)], axis=1)
        return np.ascontiguousarray(
            np.concatenate([row if j % 2 == 0 else row[::-1] for j in range(ry)], axis=0))
    ny, nx = m.phi0.shape
    return type(m)(f"{m.name}_{rx}x{ry}", tile(m.phi0), tile(m.psi0),
                   dict(m.params, nx=nx * rx, ny=ny * ry), {})


@pytest.mark.parametrize("rx,ry", [(8, 1), (1, 4), (1, 8)])
def test_factored_and_dense_directions_on_rectangles(rx, ry):
    """Directions of 2048 points and more take the factored transform (N1 x
    N2 = 32 x 64, 64 x 64, 64 x 128), shorter ones the dense product: a
    4096 x 512 grid (rows 64 x 64, columns dense), a 512 x 2048 one (rows
    dense, columns 32 x 64) and a 512 x 4096 one (columns 64 x 64), mirrored
    tiles of the 512^2 vesicle of the
    square-grid case above (the same dynamics per tile), against the FP64
    path over 60 steps at the same bound. (On tiles of a 256^2 vesicle at its
    time step the FP32 mixed path itself drifts from FP64 by 2e-5 in ten
    steps, so those grids cannot tell the transforms' rounding apart.)"""
    m = mirrored_tiles(make_workload("vesicle1024", 512)[0], rx, ry)
    note(f"gemm vs fp64 {m.params['nx']}x{m.params['ny']}")
    m0, ref = run(m, "fp64", 60, 15)
    m0g, got = run(m, "gemm", 60, 15)
    assert m0g == m0
    worst = max(max(rel_linf(g[1], r[1]), rel_linf(g[2], r[2])) for r, g in zip(ref, got))
    note(f"worst rel L-inf {worst:.3e}")
    assert worst <= 1e-6
    for g in got:
        assert abs(g[5] - m0) <= 5e-11 * abs(m0)


@pytest.mark.parametrize("rx,ry", [(32, 1), (1, 32), (128, 1), (1, 128)])
def test_factored_directions_next_to_the_narrowest_dense_one(rx, ry):
    """Strips of 2048 x 64, 64 x 2048, 8192 x 64 and 64 x 8192 cells (mirrored
    tiles of the 64^2 vesicle): a factored direction (32 x 64 or 64 x 128)
    beside a dense one of 64 points, so that every product runs its 64-wide
    tiles. Three steps against the FP64 path within 1e-6 (measured
    2.6-4.2e-8, the mixed path 3.4-4.2e-8)."""
    m = mirrored_tiles(vesicle_member(64, 43), rx, ry)
    note(f"gemm vs fp64 {m.params['nx']}x{m.params['ny']}")
    _, ref = run(m, "fp64", 3, 1)
    m0, got = run(m, "gemm", 3, 1)
    worst = max(max(rel_linf(g[1], r[1]), rel_linf(g[2], r[2])) for r, g in zip(ref, got))
    note(f"worst rel L-inf {worst:.3e}")
    assert worst <= 1e-6
    for g in got:
        assert abs(g[5] - m0) <= 5e-11 * abs(m0)


def test_gemm_variant_rejects_ensembles_graphs_and_small_grids():
    m = circle_member(32)
    with pytest.raises(C.CcmsavError) as e:
        C.Context(m.params, m.phi0, m.psi0, "gemm")      # tiles need 64 per direction
    assert e.value.name == "EUNSUPPORTED"
    with pytest.raises(C.CcmsavError) as e:
        C.Context.ensemble([m.params, m.params], [m.phi0] * 2, [m.psi0] * 2, "gemm")
    assert e.value.name == "EUNSUPPORTED"
    with pytest.raises(C.CcmsavError) as e:
        C.Context(m.params, m.phi0, m.psi0, "gemm", graph=True)
    assert e.value.name == "EUNSUPPORTED"
