"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed-form
eigenpairs (App. C), exact derivatives of the SAV functionals (Sec. 2.2),
hand-derived values on a two-cell grid, summation-by-parts identities
(App. D), the monolithic linear system of eqs. (AC_BDF2)-(Z_BDF2), the
discrete energy identity of Thm. 3.1 / App. A, exact mass conservation,
second-order temporal convergence, and symmetry invariants.
"""
import math

import numpy as np
import pytest

from oracle import ccmsav_ref as R
from oracle.monolithic import monolithic_step
from workloads import circle_member, vesicle_member


def moderate_params(nx, ny, h, **kw):
    """A parameter set where every term of the scheme has comparable weight."""
    p = dict(nx=nx, ny=ny, h=h, dt=2e-3, eps=2.0 * h, M_phi=1.0, M0=0.5,
             gamma_surf=1.0, gamma_bend=0.5, gamma_area=20.0, A=float("nan"),
             gamma_in=40.0, gamma_out=60.0, psi_in=0.3, psi_out=0.9,
             beta_in=0.2, beta_out=0.1, theta=1.5, lam=5.0, beta=0.3)
    p.update(kw)
    return p


def smooth_fields(nx, ny, h, seed=0):
    rng = np.random.default_rng(seed)
    x = (np.arange(nx) + 0.5) * h
    y = (np.arange(ny) + 0.5) * h
    X, Y = np.meshgrid(x, y)
    cx, cy = 0.5 * nx * h, 0.5 * ny * h
    r = np.hypot(X - cx, Y - cy)
    phi = np.tanh((0.3 * min(nx, ny) * h - r) / (2.0 * h))
    phi += 0.05 * rng.standard_normal(phi.shape)
    psi = 0.6 - 0.2 * phi + 0.05 * rng.standard_normal(phi.shape)
    return phi, psi


# ---------------------------------------------------------------- App. C / D

@pytest.mark.parametrize("nx,ny", [(8, 6), (5, 9)])
def test_laplacian_eigenpairs_closed_form(nx, ny):
    """Delta_h cos(pi kx (i+1/2)/nx) cos(pi ky (j+1/2)/ny) = lambda v (App. C)."""
    h = 0.37
    i = np.arange(nx) + 0.5
    j = np.arange(ny) + 0.5
    for kx in range(nx):
        for ky in range(ny):
            v = np.outer(np.cos(math.pi * ky * j / ny), np.cos(math.pi * kx * i / nx))
            lam = -(4.0 / h ** 2) * (math.sin(math.pi * kx / (2 * nx)) ** 2
                                     + math.sin(math.pi * ky / (2 * ny)) ** 2)
            np.testing.assert_allclose(R.lap(v, h), lam * v, atol=1e-12 / h ** 2)
            assert R.neumann_lap_eigs(nx, ny, h)[ky, kx] == pytest.approx(lam, rel=1e-14, abs=1e-14)


def test_laplacian_matrix_spectrum_and_symmetry():
    nx, ny, h = 6, 5, 0.5
    L = R.lap_matrix(nx, ny, h)
    np.testing.assert_allclose(L, L.T, atol=1e-13)
    ev = np.sort(np.linalg.eigvalsh(L))
    closed = np.sort(R.neumann_lap_eigs(nx, ny, h).ravel())
    np.testing.assert_allclose(ev, closed, atol=1e-11)
    # interior rows are the textbook 5-point stencil, corners see two ghosts
    c = 2 * nx + 2
    row = L[c].reshape(ny, nx)
    assert row[2, 2] == pytest.approx(-4.0 / h ** 2)
    assert row[2, 1] == row[2, 3] == row[1, 2] == row[3, 2] == pytest.approx(1.0 / h ** 2)
    assert L[0, 0] == pytest.approx(-2.0 / h ** 2)


def test_dct_matrix_is_the_normalised_cosine_basis():
    for n in (1, 2, 7, 16):
        C = R.dct_matrix(n)
        np.testing.assert_allclose(C @ C.T, np.eye(n), atol=1e-14)
        # row 0 is constant 1/sqrt(n); row k of the DCT-II basis has norm 1
        np.testing.assert_allclose(C[0], np.full(n, 1.0 / math.sqrt(n)), atol=1e-15)
    nx, ny = 8, 6
    i = np.arange(nx) + 0.5
    j = np.arange(ny) + 0.5
    v = np.outer(np.cos(math.pi * 2 * j / ny), np.cos(math.pi * 3 * i / nx))
    spec = R.dct2(v, use_matrix=True)
    expect = np.zeros((ny, nx))
    expect[2, 3] = math.sqrt(nx / 2.0) * math.sqrt(ny / 2.0)
    np.testing.assert_allclose(spec, expect, atol=1e-13)


def test_dct_round_trip_and_backends_agree():
    rng = np.random.default_rng(4)
    for shape in ((16, 16), (8, 32), (64, 48)):
        u = rng.standard_normal(shape)
        np.testing.assert_allclose(R.idct2(R.dct2(u, True), True), u, atol=1e-13)
        np.testing.assert_allclose(R.dct2(u, True), R.dct2(u, False), atol=1e-12)
        np.testing.assert_allclose(R.idct2(u, True), R.idct2(u, False), atol=1e-12)


def test_spectral_solve_equals_dense_solve():
    nx, ny, h = 7, 6, 0.4
    p = R.Params.from_dict(moderate_params(nx, ny, h))
    L = R.lap_matrix(nx, ny, h)
    rng = np.random.default_rng(1)
    f = rng.standard_normal((ny, nx))
    for alpha in (3.0 / (2 * p.dt), 1.0 / p.dt):
        C1, C2, C3 = R.chi_coefficients(p, alpha)
        chi = C1 * np.eye(nx * ny) - C2 * L + C3 * (L @ L)
        lam = R.neumann_lap_eigs(nx, ny, h)
        sigma = C1 - C2 * lam + C3 * lam ** 2
        assert sigma.min() >= C1 * (1 - 1e-15) and sigma[0, 0] == pytest.approx(C1)
        np.testing.assert_allclose(R.spectral_solve(f, sigma, True).ravel(),
                                   np.linalg.solve(chi, f.ravel()), rtol=1e-11, atol=1e-14)
        zeta = alpha * np.eye(nx * ny) - p.lam * L
        tau = alpha - p.lam * lam
        assert tau.min() >= alpha * (1 - 1e-15)
        np.testing.assert_allclose(R.spectral_solve(f, tau, True).ravel(),
                                   np.linalg.solve(zeta, f.ravel()), rtol=1e-11, atol=1e-14)


def test_summation_by_parts_and_flux_conservation():
    nx, ny, h = 9, 7, 0.3
    rng = np.random.default_rng(2)
    a, b = rng.standard_normal((2, ny, nx))
    m = 0.5 + rng.random((2, 1))
    gab = R.face_ip(R.Dx(a, h), R.Dy(a, h), R.Dx(b, h), R.Dy(b, h), h)
    assert R.ip(a, R.lap(b, h), h) == pytest.approx(-gab, rel=1e-12)
    assert R.ip(R.lap(a, h), b, h) == pytest.approx(-gab, rel=1e-12)
    mx = 0.5 + rng.random((ny, nx + 1))
    my = 0.5 + rng.random((ny + 1, nx))
    flux = R.div_mobility_grad(mx, my, b, h)
    wx, wy = np.sqrt(mx) * R.Dx(b, h), np.sqrt(my) * R.Dy(b, h)
    assert R.ip(b, flux, h) == pytest.approx(-R.face_ip(wx, wy, wx, wy, h), rel=1e-12)
    assert abs(R.integral(flux, h)) < 1e-12 * np.abs(flux).sum() * h * h
    del m


# ---------------------------------------------------------------- Sec. 2.2

def test_sav_functionals_on_constants_and_two_cells():
    nx, ny, h = 4, 3, 0.25
    p = R.Params.from_dict(moderate_params(nx, ny, h, A=0.7))
    area = nx * ny * h * h
    c, s = 0.4, 0.9
    phi = np.full((ny, nx), c)
    psi = np.full((ny, nx), s)
    assert R.sav_V(phi, p) == pytest.approx(math.sqrt(area * (c * c - 1 - p.beta) ** 2 / (4 * p.eps)))
    g = 0.25 * (c * c - 1) ** 2
    assert R.sav_U(phi, p) == pytest.approx(area * 0.75 * math.sqrt(2) * g / p.eps - 0.7)
    assert R.sav_W(phi, p) == pytest.approx(math.sqrt(area) * abs(c ** 3 - c) / p.eps)
    pc = math.sin(math.pi * c / 2)
    fin = 0.5 * p.gamma_in * (s - p.psi_in) ** 2 + p.beta_in
    fout = 0.5 * p.gamma_out * (s - p.psi_out) ** 2 + p.beta_out
    assert R.sav_Z(phi, psi, p) == pytest.approx(math.sqrt(area * ((1 + pc) * fin + (1 - pc) * fout)))
    # two cells [a, b]: one interior face, |grad|^2 of each cell = (b-a)^2/(2h^2)
    a, b = 0.2, -0.7
    two = np.array([[a, b]])
    assert R.integral(R.grad_sq_cell(two, h), h) == pytest.approx((b - a) ** 2)
    assert R.integral(6 * two ** 2 * R.grad_sq_cell(two, h), h) == pytest.approx(
        3 * (b - a) ** 2 * (a * a + b * b))
    assert R.grad_norm_sq(two, h) == pytest.approx((b - a) ** 2)


def _fd_grad(fun, u, k, delta):
    e = np.zeros_like(u)
    e.flat[k] = delta
    return (fun(u + e) - fun(u - e)) / (2 * delta)


def test_basis_functions_are_exact_discrete_gradients():
    """(1/h^2) dV/dphi_k = S_k, dU -> H, dW -> Q, dZ/dphi -> K, dZ/dpsi -> P."""
    nx, ny, h = 9, 7, 0.3
    p = R.Params.from_dict(moderate_params(nx, ny, h, A=1.3))
    phi, psi = smooth_fields(nx, ny, h, seed=3)
    S, H, Q = R.basis_S(phi, p), R.basis_H(phi, p), R.basis_Q(phi, p)
    K, P = R.basis_K(phi, psi, p), R.basis_P(phi, psi, p)
    cells = [0, nx - 1, nx * ny - 1, nx * (ny // 2) + nx // 2, 2 * nx + 1, nx + nx - 2]
    d = 1e-5
    h2 = h * h
    for k in cells:
        assert _fd_grad(lambda u: R.sav_V(u, p), phi, k, d) / h2 == pytest.approx(S.flat[k], rel=1e-7, abs=1e-8 * np.abs(S).max())
        assert _fd_grad(lambda u: R.sav_U(u, p), phi, k, d) / h2 == pytest.approx(H.flat[k], rel=1e-7, abs=1e-8 * np.abs(H).max())
        assert _fd_grad(lambda u: R.sav_W(u, p), phi, k, d) / h2 == pytest.approx(Q.flat[k], rel=1e-7, abs=1e-8 * np.abs(Q).max())
        assert _fd_grad(lambda u: R.sav_Z(u, psi, p), phi, k, d) / h2 == pytest.approx(K.flat[k], rel=1e-7, abs=1e-8 * np.abs(K).max())
        assert _fd_grad(lambda u: R.sav_Z(phi, u, p), psi, k, d) / h2 == pytest.approx(P.flat[k], rel=1e-7, abs=1e-8 * np.abs(P).max())


# ---------------------------------------------------------------- Sec. 3.2 / App. B

@pytest.mark.parametrize("shape,kw", [((6, 6), {}), ((7, 5), dict(beta=0.0, beta_in=0.0)),
                                      ((5, 4), dict(gamma_bend=2.0, theta=30.0))])
def test_step_equals_monolithic_solve(shape, kw):
    """App. B's decoupled procedure reaches the solution of eqs. (AC_BDF2)-(Z_BDF2)."""
    nx, ny = shape
    h = 0.45
    params = moderate_params(nx, ny, h, **kw)
    phi, psi = smooth_fields(nx, ny, h, seed=5)
    st = R.initial_state(phi, psi, params)
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


def _energy_identity_residuals(st_params, phi, psi, nsteps, use_matrix=True):
    st = R.initial_state(phi, psi, st_params)
    levels = []
    R.step(st, use_matrix)               # BDF1 first step
    levels.append((st.phi_prev, st.psi_prev, st.sav_prev))
    out = []
    for _ in range(nsteps):
        phi1, phi0, sav1, sav0 = st.phi, st.phi_prev, st.sav, st.sav_prev
        E_old = R.energy(st)["E"]
        info = R.step(st, use_matrix, keep=True)
        E_new = R.energy(st)["E"]
        Kn, mu_sq, cd_sq = R.dissipation_terms(st.phi, phi1, phi0, st.sav, sav1, sav0,
                                               st.psi, info["psis"], info["phis"], st.p)
        lhs = E_new - E_old + Kn
        rhs = -2.0 * st.p.dt * (st.p.M_phi * mu_sq + cd_sq)
        scale = abs(E_new) + abs(E_old) + Kn + abs(rhs)
        out.append((lhs, rhs, scale, E_new - E_old))
    return out


@pytest.mark.parametrize("kw", [{}, dict(beta=0.0, beta_in=0.0, beta_out=0.0, lam=50.0)])
def test_discrete_energy_identity_and_decay(kw):
    """E^{n+1,n} - E^{n,n-1} + K^n = -2 dt [M_phi ||mu||^2 + ||c + d/2||^2] (App. A)."""
    nx = ny = 24
    h = 0.25
    params = moderate_params(nx, ny, h, **kw)
    phi, psi = smooth_fields(nx, ny, h, seed=7)
    for lhs, rhs, scale, dE in _energy_identity_residuals(params, phi, psi, 6):
        assert abs(lhs - rhs) <= 1e-10 * scale
        assert dE <= 1e-12 * scale        # monotone decay of E_mod


def test_energy_identity_on_the_paper_parameters():
    m = circle_member(128)
    for lhs, rhs, scale, dE in _energy_identity_residuals(m.params, m.phi0, m.psi0, 5):
        assert abs(lhs - rhs) <= 1e-9 * scale
        assert dE <= 1e-12 * scale


def test_exact_mass_conservation():
    m = vesicle_member(48, 11, dt=1e-5)
    st = R.initial_state(m.phi0, m.psi0, m.params)
    m0 = R.mass(st)[0]
    for _ in range(15):
        R.step(st, use_matrix=True)
        assert abs(R.mass(st)[0] - m0) <= 1e-13 * abs(m0)


def test_second_order_in_time():
    """Cauchy errors at dt, dt/2, dt/4, dt/8 fall by about 4 (Sec. 4.1 procedure)."""
    nx = ny = 24
    h, eps, T = 0.25, 0.5, 0.002
    x = (np.arange(nx) + 0.5) * h
    X, Y = np.meshgrid(x, x)
    r = np.hypot(X - 0.52 * nx * h, (Y - 0.48 * nx * h) * 1.3)
    phi = np.tanh((0.3 * nx * h - r) / (math.sqrt(2) * eps))
    psi = 0.6 - 0.2 * phi
    sols = []
    for dt in (2e-4, 1e-4, 5e-5, 2.5e-5):
        params = moderate_params(nx, ny, h, dt=dt, eps=eps)
        st = R.run(phi, psi, params, int(round(T / dt)), use_matrix=True)
        sols.append((st.phi, st.psi))
    errs = [math.sqrt(R.ip(a[0] - b[0], a[0] - b[0], h) + R.ip(a[1] - b[1], a[1] - b[1], h))
            for a, b in zip(sols[:-1], sols[1:])]
    rates = [math.log2(e1 / e2) for e1, e2 in zip(errs[:-1], errs[1:])]
    assert all(1.9 < r < 2.1 for r in rates), rates


def test_symmetry_of_a_centred_circle_is_kept():
    m = circle_member(32, dt=1e-5)
    st = R.run(m.phi0, m.psi0, m.params, 6, use_matrix=True)
    for u in (st.phi, st.psi):
        np.testing.assert_allclose(u, u.T, atol=1e-12 * np.abs(u).max())
        np.testing.assert_allclose(u, u[::-1, :], atol=1e-12 * np.abs(u).max())
        np.testing.assert_allclose(u, u[:, ::-1], atol=1e-12 * np.abs(u).max())


def test_concentration_shift_invariance():
    """Shifting psi, psi_in, psi_out by c shifts psi and leaves phi unchanged."""
    nx = ny = 16
    h = 0.3
    params = moderate_params(nx, ny, h)
    phi, psi = smooth_fields(nx, ny, h, seed=12)
    a = R.run(phi, psi, params, 5, use_matrix=True)
    c = 0.75
    shifted = dict(params, psi_in=params["psi_in"] + c, psi_out=params["psi_out"] + c)
    b = R.run(phi, psi + c, shifted, 5, use_matrix=True)
    np.testing.assert_allclose(b.phi, a.phi, atol=1e-11)
    np.testing.assert_allclose(b.psi - c, a.psi, atol=1e-11)
    np.testing.assert_allclose(b.sav, a.sav, rtol=1e-10, atol=1e-10)


def test_oracle_catches_a_planted_sign_error(monkeypatch):
    """A plausible slip (wrong sign of the theta-tilde term) breaks the pins."""
    nx, ny = 6, 6
    h = 0.45
    params = moderate_params(nx, ny, h)
    phi, psi = smooth_fields(nx, ny, h, seed=5)
    st = R.initial_state(phi, psi, params)
    R.step(st, use_matrix=True)
    ph, _, _ = monolithic_step(st)
    monkeypatch.setattr(R, "theta_tilde", lambda p: -(p.theta + p.gamma_bend * 3 * math.sqrt(2) / (4 * p.eps)))
    old = st.phi
    R.step(st, use_matrix=True)
    assert np.abs((st.phi - old) - (ph - old)).max() > 1e-6 * np.abs(ph - old).max()


# ---------------------------------------------------------------- CC-MSAV-BDF1 (App. B remark)

def test_bdf1_scheme_steps_equal_monolithic_solve():
    """Every step of the BDF1 scheme reaches the dense solution of the BDF1
    counterparts of eqs. (AC_BDF2)-(Z_BDF2)."""
    nx, ny, h = 6, 5, 0.45
    params = moderate_params(nx, ny, h)
    phi, psi = smooth_fields(nx, ny, h, seed=9)
    st = R.initial_state(phi, psi, params, bdf1=True)
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
    # the BDF2 scheme from the same state differs after the first step
    st2 = R.run(phi, psi, params, 4, use_matrix=True)
    assert np.abs(st2.phi - st.phi).max() > 1e-6 * np.abs(st.phi - phi).max()


def test_bdf1_scheme_is_first_order_in_time():
    """Cauchy errors of the BDF1 scheme at dt, dt/2, dt/4, dt/8 fall by about 2."""
    nx = ny = 24
    h, eps, T = 0.25, 0.5, 0.002
    x = (np.arange(nx) + 0.5) * h
    X, Y = np.meshgrid(x, x)
    r = np.hypot(X - 0.52 * nx * h, (Y - 0.48 * nx * h) * 1.3)
    phi = np.tanh((0.3 * nx * h - r) / (math.sqrt(2) * eps))
    psi = 0.6 - 0.2 * phi
    sols = []
    for dt in (2e-4, 1e-4, 5e-5, 2.5e-5):
        params = moderate_params(nx, ny, h, dt=dt, eps=eps)
        st = R.run(phi, psi, params, int(round(T / dt)), use_matrix=True, bdf1=True)
        sols.append((st.phi, st.psi))
    errs = [math.sqrt(R.ip(a[0] - b[0], a[0] - b[0], h) + R.ip(a[1] - b[1], a[1] - b[1], h))
            for a, b in zip(sols[:-1], sols[1:])]
    rates = [math.log2(e1 / e2) for e1, e2 in zip(errs[:-1], errs[1:])]
    assert all(0.9 < r < 1.1 for r in rates), rates


def test_bdf1_scheme_conserves_mass_and_has_no_bdf2_energy():
    m = vesicle_member(48, 11, dt=1e-5)
    st = R.initial_state(m.phi0, m.psi0, m.params, bdf1=True)
    m0 = R.mass(st)[0]
    for _ in range(10):
        R.step(st, use_matrix=True)
        assert abs(R.mass(st)[0] - m0) <= 1e-13 * abs(m0)
    with pytest.raises(ValueError):
        R.energy(st)


# ---------------------------------------------------------------- App. F smoothing

def test_smoothing_step_equals_dense_solve():
    """One step of the App. F relaxation against the dense linear system
    (I / dt + M eps L^2) phi^1 = phi^0 / dt + (M / eps) L (phi0^3 - phi0)."""
    nx, ny, h, eps, M, dt = 6, 5, 0.3, 0.5, 0.01, 1e-3
    phi0, _ = smooth_fields(nx, ny, h, seed=3)
    phi0 = 0.5 * phi0 / np.abs(phi0).max()
    got = R.smooth_ic(phi0, h, eps, M, dt, 1, use_matrix=True, clip=False)
    L = R.lap_matrix(nx, ny, h)
    A = np.eye(nx * ny) / dt + M * eps * (L @ L)
    b = phi0.ravel() / dt + (M / eps) * (L @ (phi0.ravel() ** 3 - phi0.ravel()))
    ref = np.linalg.solve(A, b).reshape(ny, nx)
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-12)


def _sharp_disc(n, h):
    x = (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(x, x)
    return np.where(np.hypot(X - 0.5, (Y - 0.5) * 1.4) < 0.3, 1.0, -1.0)


def test_smoothing_conserves_mass_and_decreases_the_free_energy():
    n = 64
    h = 1.0 / n
    eps = 4 * h
    phi = _sharp_disc(n, h)
    mass0 = R.integral(phi, h)
    E = [R.ch_free_energy(phi, h, eps)]
    for _ in range(10):
        phi = R.smooth_ic(phi, h, eps, 0.01, 1e-6, 1, clip=False)
        E.append(R.ch_free_energy(phi, h, eps))
        assert abs(R.integral(phi, h) - mass0) <= 1e-12 * abs(mass0) + 1e-14
    assert all(b < a for a, b in zip(E[:-1], E[1:])), E
    assert E[-1] < 0.7 * E[0]
    out = R.smooth_ic(_sharp_disc(n, h), h, eps)
    assert out.min() >= -1.0 and out.max() <= 1.0


def test_smoothing_keeps_the_equilibrium_profile():
    """tanh((x - x0) / (sqrt 2 eps)) solves the steady equation, so the flow
    barely moves it, while it moves a sharp step of the same interface."""
    n = 64
    h = 1.0 / n
    eps = 4 * h
    x = (np.arange(n) + 0.5) * h
    X, _ = np.meshgrid(x, x)
    prof = np.tanh((X - 0.5) / (math.sqrt(2.0) * eps))
    step = np.where(X < 0.5, -1.0, 1.0)
    args = (h, eps, 0.01, 1e-6, 10)
    moved_prof = np.abs(R.smooth_ic(prof, *args, clip=False) - prof).max()
    moved_step = np.abs(R.smooth_ic(step, *args, clip=False) - step).max()
    assert moved_prof < 1e-3 * moved_step, (moved_prof, moved_step)


# ---------------------------------------------------------------- physical energy (Sec. 2.1)

def test_physical_energy_of_uniform_states():
    """phi = 1 everywhere: no interface, so F^surf = F^bend = 0, F^area = A^2
    gamma_area / 2, and F^osm = |Omega| f_in(psi)."""
    n, h = 16, 0.1
    params = moderate_params(n, n, h, A=0.7)
    p = R.Params.from_dict(params)
    phi = np.ones((n, n))
    psi = np.full((n, n), 0.3)
    e = R.physical_energy(phi, psi, p)
    area = (n * h) ** 2
    assert e["surf"] == 0.0 and e["bend"] == 0.0 and e["arc_length"] == 0.0
    assert math.isclose(e["area"], 0.5 * p.gamma_area * 0.7 ** 2, rel_tol=1e-14)
    f_in = 0.5 * p.gamma_in * (0.3 - p.psi_in) ** 2 + p.beta_in
    assert math.isclose(e["osm"], area * f_in, rel_tol=1e-12)
    e2 = R.physical_energy(-phi, psi, p)
    f_out = 0.5 * p.gamma_out * (0.3 - p.psi_out) ** 2 + p.beta_out
    assert math.isclose(e2["osm"], area * f_out, rel_tol=1e-12)


def test_arc_length_and_bending_energy_of_a_circle():
    """Sharp-interface limits for phi = tanh((R - r)/(sqrt2 eps)): the
    normalised surface density integrates to the perimeter 2 pi R, and the
    bending density to pi / (2 R) (kappa^2 / 4 per unit length: the 1D profile
    has int phi'^2 = 2 sqrt2 / (3 eps)); corrections are O((eps / R)^2) and,
    with about 8 cells across eps, O((h / eps)^2)."""
    n = 512
    Lbox = 2.0 * math.pi
    h = Lbox / n
    x = (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(x, x)
    R0 = 0.3 * Lbox
    eps = R0 / 20.0
    phi = np.tanh((R0 - np.hypot(X - Lbox / 2, Y - Lbox / 2)) / (math.sqrt(2.0) * eps))
    psi = np.zeros_like(phi)
    p = R.Params.from_dict(moderate_params(n, n, h, eps=eps, gamma_bend=1.0, A=0.0))
    e = R.physical_energy(phi, psi, p)
    assert abs(e["arc_length"] / (2.0 * math.pi * R0) - 1.0) < 1e-3, e["arc_length"]
    assert abs(e["bend"] / (math.pi / (2.0 * R0)) - 1.0) < 1e-2, e["bend"]


# ---------------------------------------------------------------- Dirichlet solver (App. C)

def test_dst_matrix_diagonalises_the_dirichlet_laplacian():
    """Closed form: the orthonormal DST-II rows are eigenvectors of the 1D
    Laplacian with odd ghosts, eigenvalue -(4/h^2) sin^2(pi (k+1) / 2n)."""
    n, h = 12, 0.3
    S = R.dst_matrix(n)
    np.testing.assert_allclose(S @ S.T, np.eye(n), atol=1e-14)
    L1 = np.zeros((n, n))
    for i in range(n):
        L1[i, i] = -2.0
        if i > 0:
            L1[i, i - 1] = 1.0
        if i < n - 1:
            L1[i, i + 1] = 1.0
    L1[0, 0] = L1[-1, -1] = -3.0               # ghost = minus the boundary cell
    L1 /= h * h
    lam = -(4.0 / h ** 2) * np.sin(math.pi * (np.arange(n) + 1) / (2.0 * n)) ** 2
    np.testing.assert_allclose(S @ L1 @ S.T, np.diag(lam), atol=1e-10 / h ** 2)
    from scipy.fft import dst
    x = np.random.default_rng(1).standard_normal(n)
    np.testing.assert_allclose(S @ x, dst(x, type=2, norm="ortho"), atol=1e-13)


def test_dirichlet_spectral_solve_equals_dense_solve():
    nx, ny, h = 7, 5, 0.4
    C1, C2, C3, alpha, lam = 3.0, 0.7, 0.2, 2.5, 0.9
    rhs = np.random.default_rng(2).standard_normal((ny, nx))
    L = R.lap_dirichlet_matrix(nx, ny, h)
    lam_h = R.dirichlet_lap_eigs(nx, ny, h)
    A_chi = C1 * np.eye(nx * ny) - C2 * L + C3 * (L @ L)
    A_zeta = alpha * np.eye(nx * ny) - lam * L
    for A, spec in ((A_chi, C1 - C2 * lam_h + C3 * lam_h ** 2), (A_zeta, alpha - lam * lam_h)):
        ref = np.linalg.solve(A, rhs.ravel()).reshape(ny, nx)
        for um in (True, False):
            got = R.spectral_solve_dirichlet(rhs, spec, use_matrix=um)
            np.testing.assert_allclose(got, ref, rtol=1e-11, atol=1e-12)


def test_periodic_spectral_solve_equals_dense_solve():
    """The wrap-around Laplacian's eigenvalues (closed form) and the FFT solve
    against the dense solve of chi and zeta with periodic boundaries."""
    nx, ny, h = 8, 6, 0.35
    C1, C2, C3, alpha, lam = 3.0, 0.7, 0.2, 2.5, 0.9
    L = R.lap_periodic_matrix(nx, ny, h)
    ev = np.sort(np.linalg.eigvalsh(0.5 * (L + L.T)))
    np.testing.assert_allclose(ev, np.sort(R.periodic_lap_eigs(nx, ny, h).ravel()),
                               atol=1e-10 / h ** 2)
    rhs = np.random.default_rng(3).standard_normal((ny, nx))
    lam_h = R.periodic_lap_eigs(nx, ny, h)
    for A, spec in ((C1 * np.eye(nx * ny) - C2 * L + C3 * (L @ L), C1 - C2 * lam_h + C3 * lam_h ** 2),
                    (alpha * np.eye(nx * ny) - lam * L, alpha - lam * lam_h)):
        ref = np.linalg.solve(A, rhs.ravel()).reshape(ny, nx)
        np.testing.assert_allclose(R.spectral_solve_periodic(rhs, spec), ref, rtol=1e-11,
                                   atol=1e-12)


def _three_levels(n=64):
    m = vesicle_member(n, 4)
    st = R.initial_state(m.phi0, m.psi0, m.params)
    lv = [(st.phi.copy(), st.psi.copy(), np.array(st.sav, float))]
    for _ in range(2):
        R.step(st)
        lv.append((st.phi.copy(), st.psi.copy(), np.array(st.sav, float)))
    return st.p, lv


def test_step_residuals_vanish_on_oracle_steps():
    """The discrete equations that determine a step (App. B), checked with
    stencils and inner products only, hold for the oracle's own BDF1 and BDF2
    steps to rounding: the residual check and the solve agree."""
    p, (l0, l1, l2) = _three_levels()
    for r in (R.step_residuals(*l0, *l1, p), R.step_residuals(*l1, *l2, p, *l0)):
        assert max(r.values()) <= 1e-13, r


def test_step_residuals_detect_perturbations():
    """A change of 1e-9 in phi, psi or any one SAV shows in the residuals,
    well above their rounding level (a dropped or mis-signed term gives O(1))."""
    p, (l0, l1, l2) = _three_levels()
    rng = np.random.default_rng(7)
    noise = 1e-9 * rng.standard_normal(l2[0].shape)
    assert R.step_residuals(*l1, l2[0] + noise, l2[1], l2[2], p, *l0)["chi"] >= 1e-10
    assert R.step_residuals(*l1, l2[0], l2[1] + noise, l2[2], p, *l0)["zeta"] >= 1e-10
    for i in range(4):
        sav = l2[2].copy()
        sav[i] += 1e-9 * abs(sav[i])
        assert R.step_residuals(*l1, l2[0], l2[1], sav, p, *l0)["sav"] >= 1e-12, i


@pytest.mark.parametrize("mode", ["constant", "lowest", "diagonal", "noise"])
def test_operator_inverted_residuals_recover_planted_errors(mode):
    """chi^{-1} r_phi and zeta^{-1} r_psi return an error planted in phi^{n+1}
    or psi^{n+1} at its own size, whatever its mode: the residual of
    phi^{n+1} + e is chi e (the equations are linear in the new level), so
    the operator-inverted residual is e itself, and its relative size is
    max|e| / max|phi^{n+1}| up to rounding. The spectral-radius normalised
    residual sees a constant e only at C1 / sigma_max of that size."""
    p, (l0, l1, l2) = _three_levels()
    ny, nx = l2[0].shape
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(x, y)
    shape = {"constant": np.ones((ny, nx)), "lowest": np.cos(math.pi * X),
             "diagonal": np.cos(math.pi * X) * np.cos(2 * math.pi * Y),
             "noise": np.random.default_rng(5).uniform(-1.0, 1.0, (ny, nx))}[mode]
    for which, key, key_inv in ((0, "chi", "chi_inv"), (1, "zeta", "zeta_inv")):
        amp = 1e-9 * np.abs(l2[which]).max()
        e = amp * shape / np.abs(shape).max()
        new = [l2[0], l2[1]]
        new[which] = new[which] + e
        r = R.step_residuals(*l1, new[0], new[1], l2[2], p, *l0)
        want = np.abs(e).max() / np.abs(new[which]).max()
        assert r[key_inv] == pytest.approx(want, rel=1e-3), (which, mode, r)
        if mode == "constant":
            # the spectral-radius normalisation sees the (0, 0) mode at
            # op(0) / op_max of its size: C1 / sigma_max for chi, alpha /
            # tau_max for zeta (393 and 1.8e3 at N = 4096 for the vesicle family)
            alpha = 1.5 / p.dt
            C1, C2, C3 = R.chi_coefficients(p, alpha)
            lmax = 8.0 / p.h ** 2
            ratio = (C1 / (C1 + C2 * lmax + C3 * lmax ** 2) if which == 0
                     else alpha / (alpha + p.lam * lmax))
            assert r[key] == pytest.approx(want * ratio, rel=1e-3), (which, mode, r)
