"""No kernel reads workspace memory that the step has not written first.

The library keeps every intermediate in one caller-sized workspace and never
clears most of it: the stencil output region, for one, also holds the Gram
kernel's kept spectra on grids of 8192 points per side. A read of memory
that no kernel wrote first would make a step depend on what the workspace
held before, so steps on a workspace filled with 0xFF bytes (NaN as FP32 and
FP64) must equal steps on a zeroed one bit for bit.
"""
import sys

import numpy as np
import pytest

from workloads import general_member, make_workload, vesicle_member

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2601_10057_amd import ccmsav as C  # noqa: E402


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def run(members, precision, fill, steps, graph=False):
    """Fields and SAVs of every member after ``steps`` steps on a workspace
    whose bytes all start as ``fill``."""
    params = [m.params for m in members]
    prec = C.PRECISIONS[precision]
    flags = C.FLAG_GRAPH if graph else 0
    nbytes = int(C.load().ccmsav_workspace_bytes_batch(
        len(params),
        (C.Params * len(params))(*[C.Params.from_dict(p, prec, flags) for p in params])))
    ws = torch.full((nbytes,), fill, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    out = []
    with C.Context.ensemble(params, [m.phi0 for m in members], [m.psi0 for m in members],
                            precision, workspace=ws, graph=graph) as ctx:
        ctx.step(steps)
        for i in range(len(members)):
            phi, psi = ctx.fields(i)
            s1, s0 = ctx.savs(i)
            out.append((phi, psi, np.array(s1, copy=True), np.array(s0, copy=True)))
    return out


def assert_identical(a, b, what):
    for i, (x, y) in enumerate(zip(a, b)):
        for name, u, v in zip(("phi", "psi", "sav n", "sav n-1"), x, y):
            assert np.all(np.isfinite(v)), (what, i, name)
            assert np.array_equal(u, v), (what, i, name, float(np.max(np.abs(u - v))))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("steps", [1, 3])
def test_small_grids_and_an_ensemble(precision, steps):
    members = [vesicle_member(256, 21), general_member(128, 64, 22, variant=1)]
    note(f"poisoned workspace: 256^2 + 128x64 ensemble, {precision}, {steps} steps")
    assert_identical(run(members, precision, 0, steps), run(members, precision, 255, steps),
                     "ensemble")
    note(f"poisoned workspace: 1024^2, {precision}, {steps} steps")
    single = make_workload("vesicle1024")[:1]
    assert_identical(run(single, precision, 0, steps), run(single, precision, 255, steps),
                     "vesicle1024")


def test_graph_replays_on_a_poisoned_workspace():
    members = [vesicle_member(256, 23), vesicle_member(512, 24)]
    note("poisoned workspace: 256^2 + 512^2 ensemble, mixed, graph, 4 steps")
    assert_identical(run(members, "mixed", 0, 4, graph=True),
                     run(members, "mixed", 255, 4, graph=True), "graph")


def test_n8192_mixed_with_kept_spectra_in_the_stencil_region():
    member = make_workload("vesicle8192")[:1]
    note("poisoned workspace: 8192^2 mixed, 2 steps")
    assert_identical(run(member, "mixed", 0, 2), run(member, "mixed", 255, 2), "vesicle8192")
