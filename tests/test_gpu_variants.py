"""Every combination of launch variants (row DCT band height, column-solve
and row-inverse thread shapes) gives bit-identical steps: the variants only
change how the work is split, and the two thread-count-dependent row sums use
a fixed pairwise order. ccmsav_set_launch_variants fixes the choice."""
import itertools
import sys

import numpy as np
import pytest

from workloads import vesicle_member

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2601_10057_amd import ccmsav as C  # noqa: E402


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def run(member, precision, variants, steps, graph=False):
    with C.Context(member.params, member.phi0, member.psi0, precision, graph=graph) as ctx:
        ctx.set_launch_variants(*variants)
        ctx.step(steps)
        phi, psi = ctx.fields()
        s1, s0 = ctx.savs()
        tune = ctx.tuning()
    return (phi, psi, s1, s0), tune


def rect_member():
    base = vesicle_member(64, 12)
    phi0 = np.ascontiguousarray(np.concatenate([base.phi0, base.phi0[::-1]], axis=1))
    psi0 = np.ascontiguousarray(np.concatenate([base.psi0, base.psi0[::-1]], axis=1))
    return type(base)("rect", phi0, psi0, dict(base.params, nx=128, ny=64), {})


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("shape", ["256", "rect"])
def test_all_variant_combinations_are_bit_identical(precision, shape):
    m = vesicle_member(256, 13) if shape == "256" else rect_member()
    steps = 7
    ref = None
    for combo in itertools.product((0, 1), repeat=3):
        note(f"variants {combo} {precision} {shape}")
        got, tune = run(m, precision, combo, steps)
        assert tune[0]["variants"] == dict(zip(("row_dct", "col_solve", "row_idct"), combo))
        if ref is None:
            ref = got
            continue
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), combo


def test_variants_at_the_benchmark_grid():
    m = vesicle_member(4096, 14)
    ref = None
    for combo in ((0, 0, 0), (1, 1, 1), (1, 0, 1), (0, 1, 0)):
        note(f"variants {combo} mixed 4096")
        got, _ = run(m, "mixed", combo, 3)
        if ref is None:
            ref = got
            continue
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), combo


def test_graph_replays_with_fixed_variants_and_bad_values():
    m = vesicle_member(128, 15)
    note("graph with fixed variants")
    eager, _ = run(m, "mixed", (1, 0, 1), 12)
    graph, _ = run(m, "mixed", (1, 0, 1), 12, graph=True)
    for a, b in zip(eager, graph):
        assert np.array_equal(a, b)
    with C.Context(m.params, m.phi0, m.psi0, "mixed", graph=True) as ctx:
        ctx.step(6)                                  # tuned, graph captured
        ctx.set_launch_variants(0, 1, 0)             # drops the graph
        ctx.step(6)
        phi, _ = ctx.fields()
    ref, _ = run(m, "mixed", (0, 1, 0), 12)
    assert np.array_equal(phi, ref[0])
    with C.Context(m.params, m.phi0, m.psi0) as ctx:
        for bad in ((2, 0, 0), (0, -2, 0)):
            with pytest.raises(C.CcmsavError) as e:
                ctx.set_launch_variants(*bad)
            assert e.value.name == "EINVAL"


def test_graph_replays_at_2048_match_eager_steps():
    """Grids of 2048^2 cells and more reduce the 5x5 kernel's partial rows over
    several workgroups, the last of which resets a counter for the next step;
    graph replays must repeat the eager steps bit for bit, replay after replay,
    with reads of the fields (eager work and synchronisations) in between."""
    m = vesicle_member(2048, 16)
    note("graph replays against eager steps, mixed 2048")
    with C.Context(m.params, m.phi0, m.psi0, "mixed") as e, \
            C.Context(m.params, m.phi0, m.psi0, "mixed", graph=True) as g:
        for chunk in range(4):
            e.step(3)
            g.step(3)
            pe, qe = e.fields()
            pg, qg = g.fields()
            assert np.array_equal(pe, pg), chunk
            assert np.array_equal(qe, qg), chunk
            assert np.array_equal(np.asarray(e.savs()[0]), np.asarray(g.savs()[0])), chunk
