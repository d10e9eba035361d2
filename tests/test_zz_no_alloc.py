"""ccmsav_elliptic_solve_noalloc, the allocation-free entry point, through the
C ABI: its outputs against those of ccmsav_elliptic_solve (the same solve on a
context's workspace) and against the oracle's spectral solve (App. C), on two
calls in a row with the second one smaller, in FP64 and with FP32 transforms.
Bars: 1e-12 relative L-inf in FP64 (the eigenvalue tables are formed on the
device, so the two entry points agree to rounding, not bit for bit); with
FP32 transforms 1e-6 against the context's FP32 solve."""
import ctypes
import sys

import numpy as np
import pytest

from oracle import ccmsav_ref as R
from parity_util import rel_linf
from workloads import circle_member

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2601_10057_amd import ccmsav as C  # noqa: E402


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def params_for(nx, ny):
    m = circle_member(max(nx, ny))
    return dict(m.params, nx=nx, ny=ny, A=1.0)


def context_solve(params, rhs, precision):
    """The solve of ccmsav_elliptic_solve on a fresh context of these parameters."""
    ny, nx = rhs.shape
    phi0 = np.full((ny, nx), 0.3)
    psi0 = np.full((ny, nx), 1.1)
    dev = torch.from_numpy(rhs).cuda()
    oc, oz = torch.empty_like(dev), torch.empty_like(dev)
    with C.Context(params, phi0, psi0, precision) as ctx:
        ctx.elliptic_solve(dev, oc, oz)
        torch.cuda.synchronize()
    return oc.cpu().numpy(), oz.cpu().numpy()


def oracle_solve(params, rhs):
    p = R.Params.from_dict(params)
    C1, C2, C3 = R.chi_coefficients(p, 1.5 / p.dt)
    lam = R.neumann_lap_eigs(p.nx, p.ny, p.h)
    return (R.spectral_solve(rhs, C1 - C2 * lam + C3 * lam ** 2),
            R.spectral_solve(rhs, 1.5 / p.dt - p.lam * lam))


@pytest.mark.parametrize("precision,shapes", [("fp64", [(1024, 512), (64, 32)]),
                                              ("fp64", [(1024, 1024), (16, 16)]),
                                              ("mixed", [(512, 512), (128, 64)])])
def test_noalloc_solve_matches_the_context_solve(precision, shapes):
    tol = 1e-12 if precision == "fp64" else 1e-6
    for call, (nx, ny) in enumerate(shapes):
        note(f"noalloc {precision} call {call} nx={nx} ny={ny}")
        params = params_for(nx, ny)
        rhs = np.random.default_rng(nx + 3 * ny + call).standard_normal((ny, nx))
        dev = torch.from_numpy(rhs).cuda()
        oc = torch.full_like(dev, float("nan"))
        oz = torch.full_like(dev, float("nan"))
        C.elliptic_solve_noalloc(params, dev, oc, oz, precision)
        torch.cuda.synchronize()
        got_c, got_z = oc.cpu().numpy(), oz.cpu().numpy()
        ref_c, ref_z = context_solve(params, rhs, precision)
        assert rel_linf(got_c, ref_c) <= tol, (call, rel_linf(got_c, ref_c))
        assert rel_linf(got_z, ref_z) <= tol, (call, rel_linf(got_z, ref_z))
        if precision == "fp64":
            orc, orz = oracle_solve(params, rhs)
            assert rel_linf(got_c, orc) <= 1e-12
            assert rel_linf(got_z, orz) <= 1e-12


def test_noalloc_solve_skips_a_null_output():
    nx, ny = 256, 128
    params = params_for(nx, ny)
    rhs = np.random.default_rng(5).standard_normal((ny, nx))
    dev = torch.from_numpy(rhs).cuda()
    for which in ("chi", "zeta"):
        note(f"noalloc with only {which}")
        out = torch.full_like(dev, float("nan"))
        if which == "chi":
            C.elliptic_solve_noalloc(params, dev, out, None)
        else:
            C.elliptic_solve_noalloc(params, dev, None, out)
        torch.cuda.synchronize()
        ref = oracle_solve(params, rhs)[0 if which == "chi" else 1]
        assert rel_linf(out.cpu().numpy(), ref) <= 1e-12


def test_noalloc_solve_rejects_what_it_cannot_take():
    lib = C.load()
    params = params_for(64, 64)
    rhs = torch.zeros((64, 64), dtype=torch.float64, device="cuda")
    out = torch.zeros_like(rhs)
    host = np.zeros((64, 64))
    stream = torch.cuda.current_stream().cuda_stream

    def call(p, r, a, b):
        return lib.ccmsav_elliptic_solve_noalloc(ctypes.byref(p), r, a, b, stream)

    p = C.Params.from_dict(params)
    note("noalloc error paths")
    assert call(p, None, out.data_ptr(), None) == -1                    # NULL rhs
    assert call(p, host.ctypes.data, out.data_ptr(), None) == -1        # host memory
    assert call(p, rhs.data_ptr(), host.ctypes.data, None) == -1
    big = C.Params.from_dict(params_for(2048, 64))
    assert call(big, rhs.data_ptr(), out.data_ptr(), None) == -6        # beyond 1024
    gemm = C.Params.from_dict(params, "gemm")
    assert call(gemm, rhs.data_ptr(), out.data_ptr(), None) == -6
    bad = C.Params.from_dict(dict(params, dt=-1.0))
    assert call(bad, rhs.data_ptr(), out.data_ptr(), None) == -1
    torch.cuda.synchronize()
