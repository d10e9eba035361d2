"""The fast direct solver for homogeneous Dirichlet and periodic boundaries
(ccmsav_elliptic_solve_bc: CCMSAV_BC_DIRICHLET runs the DCT kernels on the
sign-alternated input, App. C's DST form; CCMSAV_BC_PERIODIC the FFT form)
against the oracle's DST and FFT solves."""
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


def solve_case(nx, ny, precision, bc):
    m = circle_member(max(nx, ny))
    params = dict(m.params, nx=nx, ny=ny)
    rng = np.random.default_rng(nx * 31 + ny)
    rhs = rng.standard_normal((ny, nx))
    phi0 = np.zeros((ny, nx)) + 0.3
    psi0 = np.zeros((ny, nx)) + 1.1
    p = R.Params.from_dict(dict(params, A=1.0))
    C1, C2, C3 = R.chi_coefficients(p, 1.5 / p.dt)
    if bc == "dirichlet":
        lam = R.dirichlet_lap_eigs(nx, ny, p.h)
        solve = R.spectral_solve_dirichlet
    elif bc == "periodic":
        lam = R.periodic_lap_eigs(nx, ny, p.h)
        solve = R.spectral_solve_periodic
    else:
        lam = R.neumann_lap_eigs(nx, ny, p.h)
        solve = R.spectral_solve
    ref_chi = solve(rhs, C1 - C2 * lam + C3 * lam ** 2)
    ref_zeta = solve(rhs, 1.5 / p.dt - p.lam * lam)
    dev = torch.from_numpy(rhs).cuda()
    oc = torch.empty_like(dev)
    oz = torch.empty_like(dev)
    with C.Context(params, phi0, psi0, precision) as ctx:
        ctx.elliptic_solve(dev, oc, oz, bc=bc)
        torch.cuda.synchronize()
    return oc.cpu().numpy(), oz.cpu().numpy(), ref_chi, ref_zeta


@pytest.mark.parametrize("nx,ny", [(16, 16), (64, 32), (32, 128), (256, 256), (1024, 1024)])
def test_dirichlet_solves_match_oracle(nx, ny):
    note(f"dirichlet solve {nx}x{ny}")
    oc, oz, rc, rz = solve_case(nx, ny, "fp64", "dirichlet")
    assert rel_linf(oc, rc) <= 1e-12
    assert rel_linf(oz, rz) <= 1e-12


def test_dirichlet_solve_with_fp32_transforms_and_the_neumann_route():
    """FP32 transforms of a white-noise right-hand side: their rounding (unit
    u = 2^-24) spreads over all N^2 modes, while the solution is carried by
    the few low ones, so the relative error grows like N u; bound 4 N u."""
    n = 512
    note(f"dirichlet solve mixed {n}")
    oc, oz, rc, rz = solve_case(n, n, "mixed", "dirichlet")
    tol = 4 * n * 2.0 ** -24
    assert rel_linf(oc, rc) <= tol
    assert rel_linf(oz, rz) <= tol
    note("neumann through the bc entry point")
    oc, oz, rc, rz = solve_case(128, 64, "fp64", "neumann")
    assert rel_linf(oc, rc) <= 1e-12 and rel_linf(oz, rz) <= 1e-12
    # the two boundary conditions give different answers on the same input
    od, _, _, _ = solve_case(128, 64, "fp64", "dirichlet")
    assert rel_linf(od, oc) > 1e-3


def test_unknown_boundary_condition_is_rejected():
    m = circle_member(32)
    dev = torch.zeros((32, 32), dtype=torch.float64, device="cuda")
    with C.Context(m.params, m.phi0, m.psi0) as ctx:
        rc = C.load().ccmsav_elliptic_solve_bc(ctx._h, 7, dev.data_ptr(), dev.data_ptr(), None)
        assert C.STATUS.get(rc) == "EINVAL"


@pytest.mark.parametrize("nx,ny,precision", [
    (16, 16, "fp64"), (64, 32, "fp64"), (32, 128, "fp64"), (256, 256, "fp64"),
    (1024, 1024, "fp64"), (4096, 4096, "fp64"),
    (16, 16, "mixed"), (64, 32, "mixed"), (256, 256, "mixed")])
def test_periodic_solves_match_oracle(nx, ny, precision):
    """FP64 transforms in either precision of the context."""
    note(f"periodic solve {nx}x{ny} {precision}")
    oc, oz, rc, rz = solve_case(nx, ny, precision, "periodic")
    assert rel_linf(oc, rc) <= 1e-12
    assert rel_linf(oz, rz) <= 1e-12


def test_periodic_solve_of_one_output_and_its_limits():
    m = circle_member(64)
    rhs = torch.from_numpy(np.random.default_rng(5).standard_normal((64, 64))).cuda()
    oz = torch.empty_like(rhs)
    note("periodic zeta only")
    with C.Context(m.params, m.phi0, m.psi0) as ctx:
        ctx.elliptic_solve(rhs, None, oz, bc="periodic")
        torch.cuda.synchronize()
    p = R.Params.from_dict(dict(m.params, A=1.0))
    lam = R.periodic_lap_eigs(64, 64, p.h)
    ref = R.spectral_solve_periodic(rhs.cpu().numpy(), 1.5 / p.dt - p.lam * lam)
    assert rel_linf(oz.cpu().numpy(), ref) <= 1e-12
