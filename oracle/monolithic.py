"""Dense monolithic solve of one CC-MSAV step, for tiny grids.

TEST INFRASTRUCTURE ONLY (see ``ccmsav_ref``).

Eqs. (AC_BDF2)-(Z_BDF2) of Sec. 3.2 (or their BDF1 counterparts, App. B
remark, or the classical MSAV scheme's, App. B remarks) form one linear system in the 2 N^2 + 4 unknowns
(phi^{n+1}, psi^{n+1}, V^{n+1}, U^{n+1}, W^{n+1}, Z^{n+1}) once mu^{n+1} and
nu^{n+1} are substituted. This module assembles that system densely, with
Delta_h as an explicit matrix, and solves it with LU. It shares the basis
functions with the oracle but none of App. B's decoupling, so agreement with
``ccmsav_ref.step`` checks the 5x5 reduction and the DCT solves.
"""
from __future__ import annotations

import numpy as np

from . import ccmsav_ref as R


def monolithic_step(st: R.State):
    """Return (phi^{n+1}, psi^{n+1}, [V, U, W, Z]^{n+1}) without advancing ``st``."""
    p = st.p
    h, dt = p.h, p.dt
    nc = p.nx * p.ny
    L = R.lap_matrix(p.nx, p.ny, h, p.bc)
    I = np.eye(nc)
    bdf2 = st.phi_prev is not None and not st.bdf1
    phi_n, psi_n = st.phi.ravel(), st.psi.ravel()
    Vn, Un, Wn, Zn = st.sav
    if bdf2:
        phi_m, psi_m = st.phi_prev.ravel(), st.psi_prev.ravel()
        Vm, Um, Wm, Zm = st.sav_prev
        phis2 = 2.0 * st.phi - st.phi_prev
        psis2 = 2.0 * st.psi - st.psi_prev
        k_new = 3.0 / (2.0 * dt)                 # coefficient of level n+1
        rhs_phi = (4.0 * phi_n - phi_m) / (2.0 * dt)
        rhs_psi = (4.0 * psi_n - psi_m) / (2.0 * dt)
        sav_scale = 3.0
        sav_rhs = lambda old, older, F, u, uo: 4.0 * old - older + h * h * F @ (-4.0 * u + uo)  # noqa: E731
    else:
        phis2, psis2 = st.phi, st.psi
        k_new = 1.0 / dt
        rhs_phi = phi_n / dt
        rhs_psi = psi_n / dt
        sav_scale = 1.0
    phis, psis = phis2.ravel(), psis2.ravel()

    S = R.basis_S(phis2, p).ravel()
    H = R.basis_H(phis2, p).ravel()
    Q = R.basis_Q(phis2, p).ravel()
    K = R.basis_K(phis2, psis2, p).ravel()
    P = R.basis_P(phis2, psis2, p).ravel()
    mx, my = R.face_mobility(phis2, p)
    divMgradP = R.div_mobility_grad(mx, my, P.reshape(p.ny, p.nx), h, p.bc).ravel()

    sq = 3.0 * np.sqrt(2.0)
    nt = 2 * nc + 4
    A = np.zeros((nt, nt))
    b = np.zeros(nt)
    iV, iU, iW, iZ = 2 * nc, 2 * nc + 1, 2 * nc + 2, 2 * nc + 3

    # Allen-Cahn: k_new phi - (explicit) + M_phi mu^{n+1} = 0
    mu_phi = (-p.gamma_surf * sq * p.eps / 4.0 * L - p.theta * L
              + p.gamma_surf * sq * p.beta / (4.0 * p.eps) * I
              + p.gamma_bend * sq * p.eps / 8.0 * (L @ L))
    A[:nc, :nc] = k_new * I + p.M_phi * mu_phi
    A[:nc, iV] = p.M_phi * p.gamma_surf * sq / 2.0 * S
    A[:nc, iU] = p.M_phi * p.gamma_area * H
    A[:nc, iW] = p.M_phi * p.gamma_bend * sq / (8.0 * p.eps) * Q
    A[:nc, iZ] = p.M_phi * K
    b[:nc] = rhs_phi - p.M_phi * (p.theta + p.gamma_bend * sq / (4.0 * p.eps)) * (L @ phis)

    # Cahn-Hilliard: k_new psi - lambda L psi - Z div(M grad P*) = explicit - lambda L psi*;
    # in the classical scheme (App. B remarks) L is div(M_psi(phi*) grad) in both places
    if st.scheme == "classical":
        L_ch = R.div_mobility_grad_matrix(mx, my, h).toarray()
    else:
        L_ch = L
    A[nc:2 * nc, nc:2 * nc] = k_new * I - p.lam * L_ch
    A[nc:2 * nc, iZ] = -divMgradP
    b[nc:2 * nc] = rhs_psi - p.lam * (L_ch @ psis)

    # SAV equations
    for row, F, old in ((iV, S, Vn), (iU, H, Un), (iW, Q, Wn)):
        A[row, row] = sav_scale
        A[row, :nc] = -sav_scale * h * h * F
    A[iZ, iZ] = sav_scale
    A[iZ, :nc] = -sav_scale * h * h * K
    A[iZ, nc:2 * nc] = -sav_scale * h * h * P
    if bdf2:
        b[iV] = sav_rhs(Vn, Vm, S, phi_n, phi_m)
        b[iU] = sav_rhs(Un, Um, H, phi_n, phi_m)
        b[iW] = sav_rhs(Wn, Wm, Q, phi_n, phi_m)
        b[iZ] = (4.0 * Zn - Zm + h * h * K @ (-4.0 * phi_n + phi_m)
                 + h * h * P @ (-4.0 * psi_n + psi_m))
    else:
        b[iV] = Vn - h * h * S @ phi_n
        b[iU] = Un - h * h * H @ phi_n
        b[iW] = Wn - h * h * Q @ phi_n
        b[iZ] = Zn - h * h * K @ phi_n - h * h * P @ psi_n
    X = np.linalg.solve(A, b)
    return (X[:nc].reshape(p.ny, p.nx), X[nc:2 * nc].reshape(p.ny, p.nx),
            X[2 * nc:])
