"""Pins of the oracle's periodic time step (App. C names the FFT for periodic
boundaries; the scheme of Sec. 3.2 and App. B is otherwise unchanged).

With periodic boundaries every discrete operator of App. D takes wrap-around
ghosts. The step is pinned against things other than itself:
- the wrap-around Laplacian against an independent implementation by cyclic
  shifts (lap_periodic) and its closed-form Fourier eigenvalues;
- summation by parts with no boundary terms;
- the decoupled step (App. B with FFT solves) equal to the dense monolithic
  solve of eqs. (AC_BDF2)-(Z_BDF2) with the wrap-around Laplacian matrix;
- invariance under cyclic translations of the grid, which only periodic
  ghosts have (a Neumann ghost anywhere breaks it; planted below);
- exact mass conservation, and the exact discrete energy identity of App. A
  with monotone decay of the modified energy.
"""
import math

import numpy as np
import pytest

from oracle import ccmsav_ref as R
from oracle.monolithic import monolithic_step
from workloads import general_member


def periodic_params(nx, ny, h, **kw):
    p = dict(nx=nx, ny=ny, h=h, dt=2e-3, eps=2.0 * h, M_phi=0.8, M0=0.4,
             gamma_surf=1.2, gamma_bend=0.5, gamma_area=20.0, A=float("nan"),
             gamma_in=40.0, gamma_out=60.0, psi_in=0.3, psi_out=0.9,
             beta_in=0.2, beta_out=0.1, theta=1.5, lam=5.0, beta=0.3, bc="periodic")
    p.update(kw)
    return p


def blob_fields(nx, ny, h, seed=0, cx=0.37, cy=0.61):
    """A smooth periodic-friendly blob off the grid centre plus noise."""
    rng = np.random.default_rng(seed)
    x = (np.arange(nx) + 0.5) * h
    y = (np.arange(ny) + 0.5) * h
    X, Y = np.meshgrid(x, y)
    Lx, Ly = nx * h, ny * h
    dxw = np.sin(math.pi * (X - cx * Lx) / Lx) * Lx / math.pi
    dyw = np.sin(math.pi * (Y - cy * Ly) / Ly) * Ly / math.pi
    r = np.hypot(dxw, dyw)
    phi = np.tanh((0.3 * min(Lx, Ly) - r) / (2.0 * h)) + 0.05 * rng.standard_normal((ny, nx))
    psi = 0.6 - 0.2 * phi + 0.05 * rng.standard_normal((ny, nx))
    return phi, psi


def test_wraparound_laplacian_matches_cyclic_shifts_and_fourier_eigenvalues():
    nx, ny, h = 9, 6, 0.41
    u = np.random.default_rng(2).standard_normal((ny, nx))
    np.testing.assert_allclose(R.lap(u, h, "periodic"), R.lap_periodic(u, h), atol=1e-12 / h ** 2)
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    for kx in range(nx):
        for ky in range(ny):
            v = np.cos(2 * math.pi * (kx * i / nx + ky * j / ny))
            lam = -(4.0 / h ** 2) * (math.sin(math.pi * kx / nx) ** 2
                                     + math.sin(math.pi * ky / ny) ** 2)
            np.testing.assert_allclose(R.lap(v, h, "periodic"), lam * v, atol=1e-11 / h ** 2)


def test_summation_by_parts_has_no_boundary_terms():
    nx, ny, h = 8, 7, 0.3
    rng = np.random.default_rng(4)
    u, v = rng.standard_normal((ny, nx)), rng.standard_normal((ny, nx))
    mx, my = rng.uniform(0.5, 1.5, (ny, nx + 1)), rng.uniform(0.5, 1.5, (ny + 1, nx))
    mx[:, -1] = mx[:, 0]                 # one mobility per distinct face
    my[-1, :] = my[0, :]
    assert abs(R.integral(R.lap(u, h, "periodic"), h)) <= 1e-12
    lhs = R.ip(u, R.div_mobility_grad(mx, my, v, h, "periodic"), h)
    gxu, gyu = R.Dx(u, h, "periodic"), R.Dy(u, h, "periodic")
    gxv, gyv = R.Dx(v, h, "periodic"), R.Dy(v, h, "periodic")
    rhs = -R.face_ip(mx * gxu, my * gyu, gxv, gyv, h)
    assert lhs == pytest.approx(rhs, rel=1e-12)
    # a boundary face is one face: the first and last face values coincide
    np.testing.assert_allclose(gxu[:, 0], gxu[:, -1], rtol=0, atol=0)


@pytest.mark.parametrize("shape,bdf1", [((6, 6), False), ((7, 5), False), ((6, 4), True)])
def test_periodic_step_equals_monolithic_solve(shape, bdf1):
    nx, ny = shape
    h = 0.45
    params = periodic_params(nx, ny, h)
    phi, psi = blob_fields(nx, ny, h, seed=5)
    st = R.initial_state(phi, psi, params, bdf1)
    for _ in range(4):
        ph, ps, sv = monolithic_step(st)
        dphi_ref, dpsi_ref = ph - st.phi, ps - st.psi
        old_phi, old_psi = st.phi, st.psi
        R.step(st)
        np.testing.assert_allclose(st.phi - old_phi, dphi_ref, rtol=1e-8,
                                   atol=1e-10 * np.abs(dphi_ref).max())
        np.testing.assert_allclose(st.psi - old_psi, dpsi_ref, rtol=1e-8,
                                   atol=1e-10 * np.abs(dpsi_ref).max())
        np.testing.assert_allclose(st.sav, sv, rtol=1e-9, atol=1e-12)


def _run(params, phi, psi, n):
    st = R.initial_state(phi, psi, params)
    for _ in range(n):
        R.step(st)
    return st


@pytest.mark.parametrize("sx,sy", [(3, 0), (0, 5), (7, 2)])
def test_periodic_step_commutes_with_cyclic_translations(sx, sy):
    nx = ny = 16
    h = 0.3
    params = periodic_params(nx, ny, h)
    phi, psi = blob_fields(nx, ny, h, seed=9)
    a = _run(params, phi, psi, 6)
    b = _run(params, np.roll(phi, (sy, sx), (0, 1)), np.roll(psi, (sy, sx), (0, 1)), 6)
    for u, v in ((a.phi, b.phi), (a.psi, b.psi)):
        np.testing.assert_allclose(np.roll(u, (sy, sx), (0, 1)), v, atol=1e-12 * np.abs(u).max())
    np.testing.assert_allclose(a.sav, b.sav, rtol=1e-12)


def test_a_neumann_ghost_breaks_translation_invariance(monkeypatch):
    """Planted mistake: edge ghosts on the east-west faces of a periodic grid."""
    nx = ny = 16
    h = 0.3
    params = periodic_params(nx, ny, h)
    phi, psi = blob_fields(nx, ny, h, seed=9)
    orig = R.with_ghosts

    def slipped(u, bc="neumann"):
        g = orig(u, bc)
        if bc == "periodic":
            g[:, 0], g[:, -1] = g[:, 1], g[:, -2]
        return g

    monkeypatch.setattr(R, "with_ghosts", slipped)
    a = _run(params, phi, psi, 3)
    b = _run(params, np.roll(phi, 5, 1), np.roll(psi, 5, 1), 3)
    assert np.abs(np.roll(a.phi, 5, 1) - b.phi).max() > 1e-6


def test_periodic_mass_conservation_and_energy_identity():
    nx = ny = 24
    h = 0.25
    params = periodic_params(nx, ny, h)
    phi, psi = blob_fields(nx, ny, h, seed=7)
    st = R.initial_state(phi, psi, params)
    m0 = R.mass(st)[0]
    R.step(st)
    for _ in range(6):
        phi1, phi0, sav1, sav0 = st.phi, st.phi_prev, st.sav, st.sav_prev
        E_old = R.energy(st)["E"]
        info = R.step(st, keep=True)
        E_new = R.energy(st)["E"]
        Kn, mu_sq, cd_sq = R.dissipation_terms(st.phi, phi1, phi0, st.sav, sav1, sav0,
                                               st.psi, info["psis"], info["phis"], st.p)
        lhs = E_new - E_old + Kn
        rhs = -2.0 * st.p.dt * (st.p.M_phi * mu_sq + cd_sq)
        scale = abs(E_new) + abs(E_old) + Kn + abs(rhs)
        assert abs(lhs - rhs) <= 1e-10 * scale
        assert E_new - E_old <= 1e-12 * scale
        assert abs(R.mass(st)[0] - m0) <= 1e-13 * abs(m0)


def test_periodic_residual_check_vanishes_on_oracle_steps():
    m = general_member(32, 32, 10057)
    params = dict(m.params, bc="periodic")
    st = R.initial_state(m.phi0, m.psi0, params)
    lv = [(st.phi.copy(), st.psi.copy(), st.sav.copy())]
    for _ in range(2):
        R.step(st)
        lv.append((st.phi.copy(), st.psi.copy(), st.sav.copy()))
    for r in (R.step_residuals(*lv[0], *lv[1], st.p),
              R.step_residuals(*lv[1], *lv[2], st.p, *lv[0])):
        assert max(r.values()) <= 1e-13, r
