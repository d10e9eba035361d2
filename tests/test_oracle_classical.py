"""Pins of the oracle's classical MSAV scheme (App. B remarks; the comparison
system of Sec. 4), in which the Cahn-Hilliard stabilisation sits inside the
chemical potential so that zeta = alpha - lambda div(M_psi(phi*) grad) has
variable coefficients.

- The sparse operator matrix equals the stencil div(M grad) on random data.
- The decoupled step (App. B's 5x5 reduction with the variable-coefficient
  zeta solved directly) equals the dense monolithic solve of the classical
  system (BDF1 and BDF2).
- With M0 = 0 the mobility is 1, both schemes put lambda Delta_h in the same
  places, and the classical step must equal the CC step.
- The DCT-preconditioned conjugate gradient iteration (Sec. 4) reaches the
  direct solve, in a number of iterations that barely grows with the grid
  (the paper reports 12-13 per solve), and mass is conserved exactly.
"""
import numpy as np
import pytest

from oracle import ccmsav_ref as R
from oracle.monolithic import monolithic_step
from test_oracle_pins import moderate_params, smooth_fields
from workloads import vesicle_member


def test_operator_matrix_matches_the_stencil():
    nx, ny, h = 7, 5, 0.3
    rng = np.random.default_rng(3)
    mx, my = rng.uniform(0.3, 1.2, (ny, nx + 1)), rng.uniform(0.3, 1.2, (ny + 1, nx))
    u = rng.standard_normal((ny, nx))
    A = R.div_mobility_grad_matrix(mx, my, h)
    np.testing.assert_allclose((A @ u.ravel()).reshape(ny, nx), R.div_mobility_grad(mx, my, u, h),
                               rtol=1e-12, atol=1e-12 / h ** 2)
    assert abs(A - A.T).max() < 1e-12 / h ** 2                  # symmetric
    assert np.allclose(A @ np.ones(nx * ny), 0.0)               # no flux through the walls


@pytest.mark.parametrize("shape,bdf1", [((6, 6), False), ((7, 5), False), ((6, 4), True)])
def test_classical_step_equals_monolithic_solve(shape, bdf1):
    nx, ny = shape
    h = 0.45
    params = moderate_params(nx, ny, h)
    phi, psi = smooth_fields(nx, ny, h, seed=6)
    st = R.initial_state(phi, psi, params, bdf1, scheme="classical")
    for _ in range(4):
        ph, ps, sv = monolithic_step(st)
        dphi_ref, dpsi_ref = ph - st.phi, ps - st.psi
        old_phi, old_psi = st.phi, st.psi
        R.step(st, use_matrix=True)
        np.testing.assert_allclose(st.phi - old_phi, dphi_ref, rtol=1e-8,
                                   atol=1e-10 * np.abs(dphi_ref).max())
        np.testing.assert_allclose(st.psi - old_psi, dpsi_ref, rtol=1e-8,
                                   atol=1e-10 * np.abs(dpsi_ref).max())
        np.testing.assert_allclose(st.sav, sv, rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("solver", ["direct", "pcg"])
def test_classical_with_unit_mobility_is_the_cc_scheme(solver):
    m = vesicle_member(32, 7)
    params = dict(m.params, M0=0.0)
    a = R.initial_state(m.phi0, m.psi0, params)
    b = R.initial_state(m.phi0, m.psi0, params, scheme="classical", ch_solver=solver)
    for _ in range(5):
        R.step(a)
        R.step(b)
    for u, v in ((a.phi, b.phi), (a.psi, b.psi), (a.sav, b.sav)):
        assert np.abs(u - v).max() <= 1e-11 * np.abs(u).max()


def test_classical_differs_from_cc_when_the_mobility_varies():
    m = vesicle_member(32, 7)
    a = R.initial_state(m.phi0, m.psi0, m.params)
    b = R.initial_state(m.phi0, m.psi0, m.params, scheme="classical")
    for _ in range(3):
        R.step(a)
        R.step(b)
    assert np.abs(a.psi - b.psi).max() > 1e-8 * np.abs(a.psi).max()


def test_pcg_reaches_the_direct_solve_with_a_grid_independent_iteration_count():
    counts = {}
    for n in (32, 64, 128, 256):
        m = vesicle_member(n, 10057)
        d = R.initial_state(m.phi0, m.psi0, m.params, scheme="classical")
        c = R.initial_state(m.phi0, m.psi0, m.params, scheme="classical", ch_solver="pcg",
                            pcg_tol=1e-12)
        its = []
        for _ in range(3):
            R.step(d)
            its += R.step(c)["pcg_iters"]
        for u, v in ((c.phi, d.phi), (c.psi, d.psi), (c.sav, d.sav)):
            assert np.abs(u - v).max() <= 1e-11 * np.abs(v).max()
        tol10 = R.initial_state(m.phi0, m.psi0, m.params, scheme="classical", ch_solver="pcg",
                                pcg_tol=1e-10)
        counts[n] = R.step(tol10)["pcg_iters"] + R.step(tol10)["pcg_iters"]
        assert len(its) == 6 and max(its) <= 25
    allc = [k for v in counts.values() for k in v]
    assert max(allc) <= 16 and max(allc) - min(allc) <= 4, counts


@pytest.mark.parametrize("solver", ["direct", "pcg"])
def test_classical_mass_conservation(solver):
    m = vesicle_member(48, 11, dt=1e-5)
    st = R.initial_state(m.phi0, m.psi0, m.params, scheme="classical", ch_solver=solver,
                         pcg_tol=1e-8)
    m0 = R.mass(st)[0]
    for _ in range(10):
        R.step(st)
        assert abs(R.mass(st)[0] - m0) <= 1e-13 * abs(m0)
