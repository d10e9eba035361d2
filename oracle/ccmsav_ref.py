"""Plain FP64 CPU oracle of the CC-MSAV-BDF2 vesicle step.

TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the product path never does.

It follows the paper (Zhang, Li, Lowengrub & Wise, arXiv 2601.10057) as
written, in its order and notation, with numpy for array arithmetic:

* discrete operators, inner products and Neumann ghosts: App. D;
* SAV functionals V, U, W, Z: eq. (aux_vars), Sec. 2.2;
* basis functions S, H, Q, K, P: Sec. 2.2 (variational derivatives) with the
  discrete forms of Sec. 3.4.1;
* one BDF2 step: eqs. (AC_BDF2)-(Z_BDF2), solved by the procedure of App. B
  (f^n, g^n, seven elliptic solves, the 5x5 system, field recovery, SAV
  update of Algorithm 1); the first step uses the BDF1 variant of App. B,
  and a state created with ``bdf1=True`` takes every step with it (the
  CC-MSAV-BDF1 scheme of the App. B remark);
* elliptic solves: App. C (2D DCT, divide by the operator spectrum, inverse
  DCT); the DCT is the orthonormal DCT-II written out as a matrix
  (definition), with scipy's DCT as an equivalent fast library primitive for
  large grids;
* a residual check of a proposed step: the discrete equations of App. B
  that determine it (chi phi^{n+1}, zeta psi^{n+1}, the SAV relations from
  the rows of the 5x5 system), by stencils and inner products with no solve,
  for grids where a full oracle step would take minutes;
* modified discrete energy: eq. (modified_discrete_energy); the dissipation
  quantities K^n, ||mu||^2, ||c + d/2||^2 of Thm. 3.1 / App. A;
* smoothed initial conditions: App. F (constant-mobility Cahn-Hilliard
  relaxation, biharmonic term implicit, then clipping);
* homogeneous Dirichlet boundaries for the fast solver (the DST that App. C
  names for them): Laplacian with odd ghosts, DST-II matrix, eigenvalues;
  periodic boundaries (the FFT that App. C names): wrap-around Laplacian,
  eigenvalues, numpy's FFT; the whole time step with periodic boundaries
  (every operator with wrap-around ghosts, FFT solves);
* the classical MSAV scheme of the App. B remarks, the comparison system of
  Sec. 4: the Cahn-Hilliard stabilisation inside the chemical potential, so
  that zeta = alpha - lambda div(M_psi(phi*) grad) has variable coefficients;
  solved directly (sparse LU: the definition) or by the DCT-preconditioned
  conjugate gradient iteration of Sec. 4 (preconditioner alpha - lambda M_bar
  Delta_h with the spatial mean mobility M_bar, solved by App. C's DCT).

Readings where the paper is silent or ambiguous:
face mobility is M_psi of the face-averaged phi*; the face average of phi^2
in div(phi^2 grad phi) is (phi_i^2 + phi_{i+1}^2)/2; the cell |grad phi|^2
is the mean of the squared face gradients around the cell; DCTs are
orthonormal; the zero mode is divided like every other mode (its eigenvalue
is C1 > 0 or 3/(2 dt) > 0); the arc-length target A defaults to the discrete
surface energy of phi0; d^{n+1} and c^{n+1} live on faces.

Arrays are ``[ny][nx]`` (x fastest); ``u[j, i]`` is the cell (i, j).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

SQ2 = math.sqrt(2.0)

# Above this size the DCT matrix products are replaced by scipy's DCT.
MATRIX_DCT_MAX = 512


# ---------------------------------------------------------------------------
# Discrete operators on the staggered cell-centred grid (App. D)
# ---------------------------------------------------------------------------

BOUNDARIES = ("neumann", "periodic")


def with_ghosts(u: np.ndarray, bc: str = "neumann") -> np.ndarray:
    """Ghost ring of the cell-centred grid: phi_0 = phi_1, phi_{m+1} = phi_m for
    homogeneous Neumann boundaries (App. D); phi_0 = phi_m, phi_{m+1} = phi_1
    (wrap-around) for periodic ones, the case App. C pairs with the FFT."""
    if bc not in BOUNDARIES:
        raise ValueError(f"boundary condition {bc!r}")
    return np.pad(u, 1, mode="edge" if bc == "neumann" else "wrap")


def Dx(u, h, bc="neumann"):
    """(D_x u)_{i+1/2, j} on all east-west faces i = 0..m, shape (ny, nx+1)
    (with periodic boundaries faces 0 and m are the same face)."""
    g = with_ghosts(u, bc)[1:-1, :]
    return (g[:, 1:] - g[:, :-1]) / h


def Dy(u, h, bc="neumann"):
    """(D_y u)_{i, j+1/2} on all north-south faces j = 0..n, shape (ny+1, nx)."""
    g = with_ghosts(u, bc)[:, 1:-1]
    return (g[1:, :] - g[:-1, :]) / h


def Ax(u, bc="neumann"):
    """(A_x u)_{i+1/2, j} = (u_i + u_{i+1}) / 2 on east-west faces."""
    g = with_ghosts(u, bc)[1:-1, :]
    return 0.5 * (g[:, 1:] + g[:, :-1])


def Ay(u, bc="neumann"):
    """(A_y u)_{i, j+1/2} = (u_j + u_{j+1}) / 2 on north-south faces."""
    g = with_ghosts(u, bc)[:, 1:-1]
    return 0.5 * (g[1:, :] + g[:-1, :])


def dx(f, h):
    """Edge-to-centre difference (d_x f)_{i,j} = (f_{i+1/2} - f_{i-1/2}) / h."""
    return (f[:, 1:] - f[:, :-1]) / h


def dy(g, h):
    """Edge-to-centre difference (d_y g)_{i,j} = (g_{j+1/2} - g_{j-1/2}) / h."""
    return (g[1:, :] - g[:-1, :]) / h


def lap(u, h, bc="neumann"):
    """Five-point Laplacian Delta_h = d_x D_x + d_y D_y with the ghosts of bc."""
    return dx(Dx(u, h, bc), h) + dy(Dy(u, h, bc), h)


def div_mobility_grad(mob_x, mob_y, u, h, bc="neumann"):
    """d_x(M_x D_x u) + d_y(M_y D_y u) with face mobilities (Sec. 3.4.1)."""
    return dx(mob_x * Dx(u, h, bc), h) + dy(mob_y * Dy(u, h, bc), h)


def grad_sq_cell(u, h, bc="neumann"):
    """Cell value of |grad u|^2: mean of the squared face gradients (Sec. 3.4.1)."""
    gx = Dx(u, h, bc) ** 2
    gy = Dy(u, h, bc) ** 2
    return 0.5 * (gx[:, 1:] + gx[:, :-1]) + 0.5 * (gy[1:, :] + gy[:-1, :])


def ip(a, b, h):
    """Discrete L2 inner product (a, b)_h = h^2 sum a b (App. D)."""
    return h * h * float(np.sum(np.asarray(a) * np.asarray(b)))


def integral(a, h):
    """Discrete integral h^2 sum a."""
    return h * h * float(np.sum(a))


def face_ip(fx, fy, gx, gy, h):
    """[f, g]_ew + [f, g]_ns with the half-weighted two-face sums of App. D."""
    ew = 0.5 * h * h * (np.sum(fx[:, 1:] * gx[:, 1:]) + np.sum(fx[:, :-1] * gx[:, :-1]))
    ns = 0.5 * h * h * (np.sum(fy[1:, :] * gy[1:, :]) + np.sum(fy[:-1, :] * gy[:-1, :]))
    return float(ew + ns)


def grad_norm_sq(u, h, bc="neumann"):
    """||grad_h u||^2 = [D_x u, D_x u]_ew + [D_y u, D_y u]_ns (App. D)."""
    gx, gy = Dx(u, h, bc), Dy(u, h, bc)
    return face_ip(gx, gy, gx, gy, h)


def lap_matrix(nx, ny, h, bc="neumann"):
    """Dense matrix of Delta_h, built by applying the stencil to unit vectors."""
    n = nx * ny
    L = np.zeros((n, n))
    e = np.zeros((ny, nx))
    for c in range(n):
        e.flat[c] = 1.0
        L[:, c] = lap(e, h, bc).ravel()
        e.flat[c] = 0.0
    return L


# ---------------------------------------------------------------------------
# DCT and the fast direct solver (App. C)
# ---------------------------------------------------------------------------

def dct_matrix(n: int) -> np.ndarray:
    """Orthonormal DCT-II matrix C[k, i] = s_k cos(pi k (2 i + 1) / (2 n))."""
    k = np.arange(n)[:, None]
    i = np.arange(n)[None, :]
    C = np.cos(math.pi * k * (2 * i + 1) / (2.0 * n))
    C[0, :] *= math.sqrt(1.0 / n)
    C[1:, :] *= math.sqrt(2.0 / n)
    return C


_DCT_CACHE: Dict[int, np.ndarray] = {}


def _cmat(n):
    if n not in _DCT_CACHE:
        _DCT_CACHE[n] = dct_matrix(n)
    return _DCT_CACHE[n]


def dct2(u: np.ndarray, use_matrix: Optional[bool] = None) -> np.ndarray:
    """2D orthonormal DCT-II of a cell field: C_y u C_x^T."""
    ny, nx = u.shape
    if use_matrix is None:
        use_matrix = max(nx, ny) <= MATRIX_DCT_MAX
    if use_matrix:
        return _cmat(ny) @ u @ _cmat(nx).T
    from scipy.fft import dctn
    return dctn(u, type=2, norm="ortho")


def idct2(U: np.ndarray, use_matrix: Optional[bool] = None) -> np.ndarray:
    """2D orthonormal DCT-III (inverse of dct2): C_y^T U C_x."""
    ny, nx = U.shape
    if use_matrix is None:
        use_matrix = max(nx, ny) <= MATRIX_DCT_MAX
    if use_matrix:
        return _cmat(ny).T @ U @ _cmat(nx)
    from scipy.fft import idctn
    return idctn(U, type=2, norm="ortho")


def neumann_lap_eigs(nx, ny, h):
    """Eigenvalues lambda_ij of Delta_h (App. C): -(4/h^2)(sin^2(pi i/2m) + sin^2(pi j/2n)).

    Returned on the ``[ky, kx]`` grid matching ``dct2``.
    """
    lx = -(4.0 / h ** 2) * np.sin(math.pi * np.arange(nx) / (2.0 * nx)) ** 2
    ly = -(4.0 / h ** 2) * np.sin(math.pi * np.arange(ny) / (2.0 * ny)) ** 2
    return ly[:, None] + lx[None, :]


def spectral_solve(rhs, spectrum, use_matrix=None):
    """Fast direct solve of an operator diagonal in the DCT basis (App. C)."""
    return idct2(dct2(rhs, use_matrix) / spectrum, use_matrix)


# ---------------------------------------------------------------------------
# Homogeneous Dirichlet boundaries: the DST form of the fast solver (App. C)
# ---------------------------------------------------------------------------

def lap_dirichlet(u, h):
    """Five-point Laplacian with homogeneous Dirichlet ghosts: the ghost cell
    is minus its boundary neighbour (zero on the wall)."""
    ny, nx = u.shape
    g = np.zeros((ny + 2, nx + 2))
    g[1:-1, 1:-1] = u
    g[0, 1:-1], g[-1, 1:-1] = -u[0], -u[-1]
    g[1:-1, 0], g[1:-1, -1] = -u[:, 0], -u[:, -1]
    return (g[1:-1, 2:] + g[1:-1, :-2] + g[2:, 1:-1] + g[:-2, 1:-1] - 4.0 * u) / (h * h)


def lap_dirichlet_matrix(nx, ny, h):
    """Dense matrix of lap_dirichlet, built by applying it to unit vectors."""
    n = nx * ny
    L = np.zeros((n, n))
    e = np.zeros((ny, nx))
    for c in range(n):
        e.flat[c] = 1.0
        L[:, c] = lap_dirichlet(e, h).ravel()
        e.flat[c] = 0.0
    return L


def dst_matrix(n: int) -> np.ndarray:
    """Orthonormal DST-II matrix S[k, i] = s_k sin(pi (k + 1)(2 i + 1) / (2 n)),
    s_k = sqrt(2/n) except s_{n-1} = sqrt(1/n)."""
    k = np.arange(n)[:, None]
    i = np.arange(n)[None, :]
    S = np.sin(math.pi * (k + 1) * (2 * i + 1) / (2.0 * n)) * math.sqrt(2.0 / n)
    S[-1, :] *= math.sqrt(0.5)
    return S


def dirichlet_lap_eigs(nx, ny, h):
    """Eigenvalues of lap_dirichlet on the ``[ky, kx]`` grid of the DST-II:
    -(4/h^2)(sin^2(pi (i+1)/2m) + sin^2(pi (j+1)/2n))."""
    lx = -(4.0 / h ** 2) * np.sin(math.pi * (np.arange(nx) + 1) / (2.0 * nx)) ** 2
    ly = -(4.0 / h ** 2) * np.sin(math.pi * (np.arange(ny) + 1) / (2.0 * ny)) ** 2
    return ly[:, None] + lx[None, :]


def spectral_solve_dirichlet(rhs, spectrum, use_matrix=None):
    """Fast direct solve of an operator diagonal in the DST-II basis (the
    Dirichlet counterpart of App. C's DCT solver)."""
    ny, nx = rhs.shape
    if use_matrix is None:
        use_matrix = max(nx, ny) <= MATRIX_DCT_MAX
    if use_matrix:
        Sy, Sx = dst_matrix(ny), dst_matrix(nx)
        return Sy.T @ ((Sy @ rhs @ Sx.T) / spectrum) @ Sx
    from scipy.fft import dstn, idstn
    return idstn(dstn(rhs, type=2, norm="ortho") / spectrum, type=2, norm="ortho")


# ---------------------------------------------------------------------------
# Periodic boundaries: the FFT form of the fast solver (App. C)
# ---------------------------------------------------------------------------

def lap_periodic(u, h):
    """Five-point Laplacian with periodic wrap-around."""
    return (np.roll(u, 1, 1) + np.roll(u, -1, 1) + np.roll(u, 1, 0) + np.roll(u, -1, 0)
            - 4.0 * u) / (h * h)


def lap_periodic_matrix(nx, ny, h):
    """Dense matrix of lap_periodic, built by applying it to unit vectors."""
    n = nx * ny
    L = np.zeros((n, n))
    e = np.zeros((ny, nx))
    for c in range(n):
        e.flat[c] = 1.0
        L[:, c] = lap_periodic(e, h).ravel()
        e.flat[c] = 0.0
    return L


def periodic_lap_eigs(nx, ny, h):
    """Eigenvalues of lap_periodic on the ``[ky, kx]`` grid of the 2D DFT:
    -(4/h^2)(sin^2(pi i/m) + sin^2(pi j/n))."""
    lx = -(4.0 / h ** 2) * np.sin(math.pi * np.arange(nx) / nx) ** 2
    ly = -(4.0 / h ** 2) * np.sin(math.pi * np.arange(ny) / ny) ** 2
    return ly[:, None] + lx[None, :]


def spectral_solve_periodic(rhs, spectrum):
    """Fast direct solve of an operator diagonal in the Fourier basis (the
    periodic counterpart of App. C's DCT solver), with numpy's FFT."""
    return np.real(np.fft.ifft2(np.fft.fft2(rhs) / spectrum))


def lap_eigs(p: "Params"):
    """Eigenvalues of Delta_h for the boundary conditions of p, on the grid of
    the transform that diagonalises it (DCT-II for Neumann, DFT for periodic)."""
    if p.bc == "periodic":
        return periodic_lap_eigs(p.nx, p.ny, p.h)
    return neumann_lap_eigs(p.nx, p.ny, p.h)


def fast_solve(rhs, spectrum, p: "Params", use_matrix=None):
    """App. C's fast direct solve with the transform of p's boundary conditions."""
    if p.bc == "periodic":
        return spectral_solve_periodic(rhs, spectrum)
    return spectral_solve(rhs, spectrum, use_matrix)


# ---------------------------------------------------------------------------
# Model pieces (Sec. 2)
# ---------------------------------------------------------------------------

@dataclass
class Params:
    nx: int
    ny: int
    h: float
    dt: float
    eps: float
    M_phi: float
    M0: float
    gamma_surf: float
    gamma_bend: float
    gamma_area: float
    A: float
    gamma_in: float
    gamma_out: float
    psi_in: float
    psi_out: float
    beta_in: float
    beta_out: float
    theta: float
    lam: float
    beta: float
    bc: str = "neumann"      # "neumann" (App. D) or "periodic"

    @classmethod
    def from_dict(cls, d: Dict) -> "Params":
        names = [k for k in cls.__dataclass_fields__ if k != "bc"]
        return cls(**{k: d[k] for k in names}, bc=d.get("bc", "neumann"))


def p_interp(phi):
    """Interpolation p(phi) = sin(pi phi / 2) (Sec. 2.1)."""
    return np.sin(0.5 * math.pi * phi)


def dp_interp(phi):
    """p'(phi) = (pi/2) cos(pi phi / 2)."""
    return 0.5 * math.pi * np.cos(0.5 * math.pi * phi)


def f_in(psi, p: Params):
    """f^in(psi) = gamma_in/2 (psi - psi_in)^2 + beta_in (Sec. 2.1)."""
    return 0.5 * p.gamma_in * (psi - p.psi_in) ** 2 + p.beta_in


def f_out(psi, p: Params):
    """f^out(psi) = gamma_out/2 (psi - psi_out)^2 + beta_out (Sec. 2.1)."""
    return 0.5 * p.gamma_out * (psi - p.psi_out) ** 2 + p.beta_out


def mobility_psi(phi, p: Params):
    """Cahn-Hilliard mobility M_psi(phi) = 1 - M0 (phi^2 - 1)^2 (Sec. 2.1)."""
    return 1.0 - p.M0 * (phi * phi - 1.0) ** 2


def double_well(phi):
    """g(phi) = (phi^2 - 1)^2 / 4."""
    return 0.25 * (phi * phi - 1.0) ** 2


def f_surf(phi, p: Params):
    """Surface density (3 sqrt2/4)(g/eps + eps/2 |grad phi|^2), cell form."""
    return 0.75 * SQ2 * (double_well(phi) / p.eps
                         + 0.5 * p.eps * grad_sq_cell(phi, p.h, p.bc))


def sav_V(phi, p: Params):
    """V = sqrt(int (phi^2 - 1 - beta)^2 / (4 eps)) (eq. aux_VW)."""
    return math.sqrt(integral((phi * phi - 1.0 - p.beta) ** 2 / (4.0 * p.eps), p.h))


def sav_U(phi, p: Params):
    """U = int f_surf - A (eq. aux_ZU)."""
    return integral(f_surf(phi, p), p.h) - p.A


def w_density(phi, p: Params):
    """Integrand of W^2: 6 phi^2 |grad phi|^2 + (phi^3 - phi)^2 / eps^2."""
    return (6.0 * phi * phi * grad_sq_cell(phi, p.h, p.bc)
            + (phi ** 3 - phi) ** 2 / p.eps ** 2)


def sav_W(phi, p: Params):
    """W = sqrt(int w_density) (eq. aux_VW)."""
    return math.sqrt(integral(w_density(phi, p), p.h))


def osm_twice(phi, psi, p: Params):
    """2 f_osm = (1 + p) f_in + (1 - p) f_out (eq. osm_density)."""
    pp = p_interp(phi)
    return (1.0 + pp) * f_in(psi, p) + (1.0 - pp) * f_out(psi, p)


def sav_Z(phi, psi, p: Params):
    """Z = sqrt(2 int f_osm) (eq. aux_ZU)."""
    return math.sqrt(integral(osm_twice(phi, psi, p), p.h))


def basis_S(phi, p: Params):
    """S(phi) = phi (phi^2 - 1 - beta)/eps / (2 sqrt(int (phi^2-1-beta)^2/(4 eps)))."""
    return (phi * (phi * phi - 1.0 - p.beta) / p.eps) / (2.0 * sav_V(phi, p))


def basis_H(phi, p: Params):
    """H(phi) = (3 sqrt2/4)(phi (phi^2 - 1)/eps - eps Delta_h phi)."""
    return 0.75 * SQ2 * (phi * (phi * phi - 1.0) / p.eps - p.eps * lap(phi, p.h, p.bc))


def basis_Q(phi, p: Params):
    """Q(phi) = {6 [phi|grad phi|^2 - div(phi^2 grad phi)] + (phi^3-phi)(3phi^2-1)/eps^2} / W.

    [phi |grad phi|^2] and [div(phi^2 grad phi)] follow Sec. 3.4.1 with the
    face average of phi^2 taken as (phi_i^2 + phi_{i+1}^2)/2.
    """
    h, bc = p.h, p.bc
    sq = phi * phi
    term_a = phi * grad_sq_cell(phi, h, bc)
    term_b = dx(Ax(sq, bc) * Dx(phi, h, bc), h) + dy(Ay(sq, bc) * Dy(phi, h, bc), h)
    num = 6.0 * (term_a - term_b) + (phi ** 3 - phi) * (3.0 * sq - 1.0) / p.eps ** 2
    return num / sav_W(phi, p)


def basis_K(phi, psi, p: Params):
    """K = p'(phi)(f_in - f_out) / (2 sqrt(int[(1+p) f_in + (1-p) f_out]))."""
    return dp_interp(phi) * (f_in(psi, p) - f_out(psi, p)) / (2.0 * sav_Z(phi, psi, p))


def basis_P(phi, psi, p: Params):
    """P = [gamma_in (1+p)(psi - psi_in) + gamma_out (1-p)(psi - psi_out)] / (2 Z)."""
    pp = p_interp(phi)
    num = (p.gamma_in * (1.0 + pp) * (psi - p.psi_in)
           + p.gamma_out * (1.0 - pp) * (psi - p.psi_out))
    return num / (2.0 * sav_Z(phi, psi, p))


def face_mobility(phi, p: Params):
    """M_psi evaluated at the face-averaged phi (Sec. 3.4.1)."""
    return mobility_psi(Ax(phi, p.bc), p), mobility_psi(Ay(phi, p.bc), p)


# ---------------------------------------------------------------------------
# Time stepping (Sec. 3.2 and App. B)
# ---------------------------------------------------------------------------

@dataclass
class State:
    """Two time levels of the fields plus the SAVs and the energy accumulator."""
    p: Params
    phi: np.ndarray              # level n
    psi: np.ndarray
    phi_prev: Optional[np.ndarray]   # level n-1 (None before the first step)
    psi_prev: Optional[np.ndarray]
    sav: np.ndarray              # (V, U, W, Z) at level n
    sav_prev: Optional[np.ndarray]
    n: int = 0
    d_acc: float = 0.0           # sum_{j>=2} (dt/2) ||d^j||^2
    history: List[Dict] = field(default_factory=list)
    bdf1: bool = False           # every step with the BDF1 scheme
    scheme: str = "cc"           # "cc", or "classical" (App. B remarks)
    ch_solver: str = "direct"    # classical zeta solves: "direct" or "pcg"
    pcg_tol: float = 1e-12       # relative residual at which PCG stops
    pcg_maxit: int = 200


def initial_state(phi0, psi0, params: Dict, bdf1: bool = False, scheme: str = "cc",
                  ch_solver: str = "direct", pcg_tol: float = 1e-12,
                  pcg_maxit: int = 200) -> State:
    """Initial fields and SAVs (eq. msav_ic); A defaults to int f_surf(phi0).
    With ``bdf1`` every step uses the CC-MSAV-BDF1 scheme (App. B remark).
    ``scheme="classical"`` takes the classical MSAV scheme instead (App. B
    remarks), its variable-coefficient zeta solved by ``ch_solver``."""
    p = Params.from_dict(params)
    phi0 = np.array(phi0, dtype=np.float64)
    psi0 = np.array(psi0, dtype=np.float64)
    if not math.isfinite(p.A):
        p.A = integral(f_surf(phi0, p), p.h)
    sav = np.array([sav_V(phi0, p), sav_U(phi0, p), sav_W(phi0, p),
                    sav_Z(phi0, psi0, p)])
    if scheme not in ("cc", "classical") or ch_solver not in ("direct", "pcg"):
        raise ValueError(f"scheme {scheme!r}, solver {ch_solver!r}")
    if scheme == "classical" and p.bc != "neumann":
        raise ValueError("the classical scheme is taken with Neumann boundaries")
    return State(p, phi0, psi0, None, None, sav, None, bdf1=bdf1, scheme=scheme,
                 ch_solver=ch_solver, pcg_tol=pcg_tol, pcg_maxit=pcg_maxit)


def chi_coefficients(p: Params, alpha: float):
    """C1, C2, C3 of the Allen-Cahn operator chi (App. B, Step 3)."""
    C1 = alpha + p.M_phi * p.gamma_surf * 3.0 * SQ2 * p.beta / (4.0 * p.eps)
    C2 = p.M_phi * (p.gamma_surf * 3.0 * SQ2 * p.eps / 4.0 + p.theta)
    C3 = p.M_phi * p.gamma_bend * 3.0 * SQ2 * p.eps / 8.0
    return C1, C2, C3


def theta_tilde(p: Params):
    """theta + gamma_bend 3 sqrt2 / (4 eps) (Sec. 3.3)."""
    return p.theta + p.gamma_bend * 3.0 * SQ2 / (4.0 * p.eps)


def sav_weights(p: Params):
    """c_gs, c_ga, c_gb, c_go of App. B, Step 3."""
    return (p.M_phi * p.gamma_surf * 3.0 * SQ2 / 2.0,
            p.M_phi * p.gamma_area,
            p.M_phi * p.gamma_bend * 3.0 * SQ2 / (8.0 * p.eps),
            p.M_phi)


# ---------------------------------------------------------------------------
# The classical MSAV scheme's Cahn-Hilliard operator (App. B remarks, Sec. 4)
# ---------------------------------------------------------------------------

def div_mobility_grad_matrix(mx, my, h):
    """Sparse matrix of u -> div(M grad u) = d_x(M_x D_x u) + d_y(M_y D_y u)
    with Neumann ghosts (the wall faces carry no flux), for face mobilities
    mx (ny, nx+1) and my (ny+1, nx)."""
    import scipy.sparse as sp
    ny, nx = mx.shape[0], my.shape[1]
    ie = mx[:, 1:].copy()            # east face of cell (i, j)
    iw = mx[:, :-1].copy()           # west face
    jn = my[1:, :].copy()            # north face
    js = my[:-1, :].copy()           # south face
    ie[:, -1] = 0.0
    iw[:, 0] = 0.0
    jn[-1, :] = 0.0
    js[0, :] = 0.0
    diag = -(ie + iw + jn + js).ravel()
    n = nx * ny
    A = sp.diags([diag, ie.ravel()[:-1], iw.ravel()[1:], jn.ravel()[:-nx], js.ravel()[nx:]],
                 [0, 1, -1, nx, -nx], shape=(n, n), format="csr")
    return A / (h * h)


def pcg(apply_A, b, apply_Pinv, tol, maxit, h):
    """Preconditioned conjugate gradients (Hestenes-Stiefel form) from x = 0
    for a symmetric positive definite A, stopping when the discrete L2 norm of
    the residual is at most tol times that of b. Returns (x, iterations)."""
    x = np.zeros_like(b)
    r = b.copy()
    bnorm = math.sqrt(ip(b, b, h))
    if bnorm == 0.0:
        return x, 0
    z = apply_Pinv(r)
    p = z.copy()
    rz = ip(r, z, h)
    for it in range(1, maxit + 1):
        q = apply_A(p)
        a = rz / ip(p, q, h)
        x = x + a * p
        r = r - a * q
        if math.sqrt(ip(r, r, h)) <= tol * bnorm:
            return x, it
        z = apply_Pinv(r)
        rz_new = ip(r, z, h)
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, maxit


def classical_zeta_solver(st: "State", mx, my, alpha: float, phis):
    """The classical scheme's zeta^{-1} for this step: zeta = alpha -
    lambda div(M grad) with the face mobilities of phi*. Direct: sparse LU
    (the definition). PCG (Sec. 4): the preconditioner alpha - lambda M_bar
    Delta_h, M_bar the spatial mean of M_psi(phi*) over the cells, solved by
    App. C's DCT; afterwards the mean of the iterate is set to the exact
    mean(b) / alpha (summing zeta x = b over the cells gives alpha sum x =
    sum b, since the fluxes cancel), so that mass is conserved to rounding
    whatever the residual. Returns (solve, iteration counts)."""
    p = st.p
    h = p.h
    n = p.nx * p.ny
    iters = []
    if st.ch_solver == "direct":
        import scipy.sparse as sp
        from scipy.sparse.linalg import splu
        A = sp.identity(n, format="csc") * alpha - p.lam * div_mobility_grad_matrix(mx, my, h).tocsc()
        lu = splu(A.tocsc())
        return (lambda r: lu.solve(r.ravel()).reshape(p.ny, p.nx)), iters
    m_bar = float(np.mean(mobility_psi(phis, p)))
    spectrum = alpha - p.lam * m_bar * neumann_lap_eigs(p.nx, p.ny, h)
    apply_A = lambda u: alpha * u - p.lam * div_mobility_grad(mx, my, u, h)   # noqa: E731
    apply_P = lambda r: spectral_solve(r, spectrum)                           # noqa: E731

    def solve(b):
        x, it = pcg(apply_A, b, apply_P, st.pcg_tol, st.pcg_maxit, h)
        iters.append(it)
        return x + (np.sum(b) / alpha - np.sum(x)) / n
    return solve, iters


def step(st: State, use_matrix: Optional[bool] = None, keep: bool = False) -> Dict:
    """Advance one step: BDF1 variant first (App. B remark), BDF2 after (or
    BDF1 throughout for a state of the BDF1 scheme).

    Returns a dict of intermediate quantities (the 5x5 system, etc.).
    """
    p = st.p
    h, dt = p.h, p.dt
    bdf2 = st.phi_prev is not None and not st.bdf1
    phi_n, psi_n = st.phi, st.psi
    Vn, Un, Wn, Zn = st.sav
    if bdf2:
        phi_m, psi_m = st.phi_prev, st.psi_prev
        Vm, Um, Wm, Zm = st.sav_prev
        phis = 2.0 * phi_n - phi_m
        psis = 2.0 * psi_n - psi_m
        alpha = 3.0 / (2.0 * dt)
    else:
        phis, psis = phi_n, psi_n
        alpha = 1.0 / dt

    S = basis_S(phis, p)
    H = basis_H(phis, p)
    Q = basis_Q(phis, p)
    K = basis_K(phis, psis, p)
    P = basis_P(phis, psis, p)
    mx, my = face_mobility(phis, p)
    LP_src = div_mobility_grad(mx, my, P, h, p.bc)    # div(M_psi(phi*) grad P*)

    # Bracketed explicit SAV parts: BDF2 carries the 1/3 of the paper's f^n.
    if bdf2:
        dphi = -4.0 * phi_n + phi_m
        dpsi = -4.0 * psi_n + psi_m
        sV = (4.0 * Vn - Vm + ip(S, dphi, h)) / 3.0
        sU = (4.0 * Un - Um + ip(H, dphi, h)) / 3.0
        sW = (4.0 * Wn - Wm + ip(Q, dphi, h)) / 3.0
        sZ = (4.0 * Zn - Zm + ip(K, dphi, h) + ip(P, dpsi, h)) / 3.0
        a_phi = (4.0 * phi_n - phi_m) / (2.0 * dt)
        a_psi = (4.0 * psi_n - psi_m) / (2.0 * dt)
    else:
        sV = Vn + ip(S, -phi_n, h)
        sU = Un + ip(H, -phi_n, h)
        sW = Wn + ip(Q, -phi_n, h)
        sZ = Zn + ip(K, -phi_n, h) + ip(P, -psi_n, h)
        a_phi = phi_n / dt
        a_psi = psi_n / dt

    tt = theta_tilde(p)
    f = a_phi - p.M_phi * (tt * lap(phis, h, p.bc)
                           + p.gamma_surf * 1.5 * SQ2 * sV * S
                           + p.gamma_area * sU * H
                           + p.gamma_bend * 3.0 * SQ2 / (8.0 * p.eps) * sW * Q
                           + sZ * K)
    nu_tilde = sZ * P
    classical = st.scheme == "classical"
    if classical:
        # the stabilisation inside the chemical potential (App. B remarks):
        # g = b^n + div(M grad(-lambda psi* + s_Z P))
        g = a_psi + div_mobility_grad(mx, my, -p.lam * psis + nu_tilde, h, p.bc)
    else:
        g = a_psi - p.lam * lap(psis, h, p.bc) + div_mobility_grad(mx, my, nu_tilde, h, p.bc)

    C1, C2, C3 = chi_coefficients(p, alpha)
    lam_h = lap_eigs(p)
    sigma = C1 - C2 * lam_h + C3 * lam_h ** 2
    tau = alpha - p.lam * lam_h

    chi_inv = lambda r: fast_solve(r, sigma, p, use_matrix)   # noqa: E731
    pcg_iters = []
    if classical:
        zeta_inv, pcg_iters = classical_zeta_solver(st, mx, my, alpha, phis)
    else:
        zeta_inv = lambda r: fast_solve(r, tau, p, use_matrix)    # noqa: E731
    f_hat = chi_inv(f)
    S_hat, H_hat, Q_hat, K_hat = chi_inv(S), chi_inv(H), chi_inv(Q), chi_inv(K)
    g_hat = zeta_inv(g)
    Lam_P = zeta_inv(LP_src)

    cgs, cga, cgb, cgo = sav_weights(p)
    F = [S, H, Q, K]
    Fh = [S_hat, H_hat, Q_hat, K_hat]
    cw = [cgs, cga, cgb, cgo]
    M = np.zeros((5, 5))
    b = np.zeros(5)
    for i in range(4):
        for j in range(4):
            M[i, j] = cw[j] * ip(F[i], Fh[j], h) + (1.0 if i == j else 0.0)
        M[i, 4] = cgo * ip(F[i], K_hat, h)
        b[i] = ip(F[i], f_hat, h)
    PL = ip(P, Lam_P, h)
    M[4, 3] = -PL
    M[4, 4] = 1.0 - PL
    b[4] = ip(P, g_hat, h)
    x = np.linalg.solve(M, b)
    B, C, D, E, G = x

    phi_new = f_hat - cgs * B * S_hat - cga * C * H_hat - cgb * D * Q_hat \
        - cgo * (E + G) * K_hat
    psi_new = g_hat + (E + G) * Lam_P
    sav_new = np.array([B + sV, C + sU, D + sW, E + G + sZ])

    info = dict(bdf2=bdf2, M=M, b=b, x=x, s=np.array([sV, sU, sW, sZ]),
                norms=np.array([sav_V(phis, p), sav_W(phis, p), sav_Z(phis, psis, p)]),
                pcg_iters=list(pcg_iters))
    if keep:
        info.update(S=S, H=H, Q=Q, K=K, P=P, LP=LP_src, f=f, g=g,
                    phis=phis, psis=psis, sigma=sigma, tau=tau)

    if bdf2 and not classical:
        st.d_acc += 0.5 * dt * d_norm_sq(psi_new, psis, phis, p)
    st.phi_prev, st.psi_prev, st.sav_prev = phi_n, psi_n, st.sav
    st.phi, st.psi, st.sav = phi_new, psi_new, sav_new
    st.n += 1
    return info


def step_residuals(phi_n, psi_n, sav_n, phi_new, psi_new, sav_new, p: Params,
                   phi_m=None, psi_m=None, sav_m=None) -> Dict:
    """How far a proposed step result is from the step's discrete equations.

    The BDF2 step (BDF1 when no level n-1 is given) of App. B is the unique
    solution of, with x = (B, C, D, E + G) = (V, U, W, Z)^{n+1} minus the
    bracketed explicit SAV parts:
      chi phi^{n+1} = f - c_gs B S - c_ga C H - c_gb D Q - c_go (E + G) K,
      zeta psi^{n+1} = g + (E + G) div(M grad P),
      B = (S, phi^{n+1}), C = (H, phi^{n+1}), D = (Q, phi^{n+1}),
      E + G = (K, phi^{n+1}) + (P, psi^{n+1}),
    where the last four follow from the 5x5 system's rows. Checking them needs
    stencils and inner products only (no solve), at any grid size.

    Returns relative residuals: ``chi`` = max|chi phi - rhs| over
    sigma_max max|phi|, ``zeta`` likewise with tau_max, ``sav`` = the largest
    |x_i - (F_i, .)| over (|F_i|, |.|). The first two weigh every mode by the
    largest eigenvalue of the operator, so a smooth error (weighted by sigma
    near C1 and tau near alpha) shows sigma_max / C1 times smaller than it is.
    ``chi_inv`` = max|chi^{-1} r_phi| / max|phi^{n+1}| and ``zeta_inv`` =
    max|zeta^{-1} r_psi| / max|psi^{n+1}| map the residuals back through the
    operators (App. C's spectral solve): chi^{-1} r_phi is the change of
    phi^{n+1} that the residual stands for, in every mode alike.
    """
    h, dt = p.h, p.dt
    bdf2 = phi_m is not None
    if bdf2:
        phis, psis = 2.0 * phi_n - phi_m, 2.0 * psi_n - psi_m
        alpha = 3.0 / (2.0 * dt)
    else:
        phis, psis = phi_n, psi_n
        alpha = 1.0 / dt
    S, H, Q = basis_S(phis, p), basis_H(phis, p), basis_Q(phis, p)
    K, P = basis_K(phis, psis, p), basis_P(phis, psis, p)
    mx, my = face_mobility(phis, p)
    LP_src = div_mobility_grad(mx, my, P, h, p.bc)
    Vn, Un, Wn, Zn = sav_n
    if bdf2:
        Vm, Um, Wm, Zm = sav_m
        dphi, dpsi = -4.0 * phi_n + phi_m, -4.0 * psi_n + psi_m
        s = [(4.0 * Vn - Vm + ip(S, dphi, h)) / 3.0, (4.0 * Un - Um + ip(H, dphi, h)) / 3.0,
             (4.0 * Wn - Wm + ip(Q, dphi, h)) / 3.0,
             (4.0 * Zn - Zm + ip(K, dphi, h) + ip(P, dpsi, h)) / 3.0]
        a_phi, a_psi = (4.0 * phi_n - phi_m) / (2.0 * dt), (4.0 * psi_n - psi_m) / (2.0 * dt)
    else:
        s = [Vn - ip(S, phi_n, h), Un - ip(H, phi_n, h), Wn - ip(Q, phi_n, h),
             Zn - ip(K, phi_n, h) - ip(P, psi_n, h)]
        a_phi, a_psi = phi_n / dt, psi_n / dt
    tt = theta_tilde(p)
    f = a_phi - p.M_phi * (tt * lap(phis, h, p.bc) + p.gamma_surf * 1.5 * SQ2 * s[0] * S
                           + p.gamma_area * s[1] * H
                           + p.gamma_bend * 3.0 * SQ2 / (8.0 * p.eps) * s[2] * Q + s[3] * K)
    g = a_psi - p.lam * lap(psis, h, p.bc) + div_mobility_grad(mx, my, s[3] * P, h, p.bc)
    x = [sav_new[i] - s[i] for i in range(4)]
    cgs, cga, cgb, cgo = sav_weights(p)
    C1, C2, C3 = chi_coefficients(p, alpha)
    L_phi = lap(phi_new, h, p.bc)
    r_phi = (C1 * phi_new - C2 * L_phi + C3 * lap(L_phi, h, p.bc)
             - (f - cgs * x[0] * S - cga * x[1] * H - cgb * x[2] * Q - cgo * x[3] * K))
    r_psi = alpha * psi_new - p.lam * lap(psi_new, h, p.bc) - (g + x[3] * LP_src)
    lmax = 8.0 / (h * h)                                # spectral radius of -Delta_h
    sig_max = abs(C1) + abs(C2) * lmax + abs(C3) * lmax * lmax
    tau_max = alpha + abs(p.lam) * lmax
    aphi, apsi = np.abs(phi_new), np.abs(psi_new)
    sav = 0.0
    for xi, F in zip(x[:3], (S, H, Q)):
        sav = max(sav, abs(xi - ip(F, phi_new, h)) / ip(np.abs(F), aphi, h))
    sav = max(sav, abs(x[3] - ip(K, phi_new, h) - ip(P, psi_new, h))
              / (ip(np.abs(K), aphi, h) + ip(np.abs(P), apsi, h)))
    lam_h = lap_eigs(p)
    e_phi = fast_solve(r_phi, C1 - C2 * lam_h + C3 * lam_h ** 2, p)
    e_psi = fast_solve(r_psi, alpha - p.lam * lam_h, p)
    return dict(chi=float(np.max(np.abs(r_phi)) / (sig_max * np.max(aphi))),
                zeta=float(np.max(np.abs(r_psi)) / (tau_max * np.max(apsi))),
                sav=float(sav),
                chi_inv=float(np.max(np.abs(e_phi)) / np.max(aphi)),
                zeta_inv=float(np.max(np.abs(e_psi)) / np.max(apsi)))


def run(phi0, psi0, params: Dict, nsteps: int, use_matrix=None, bdf1: bool = False) -> State:
    """Initialise and take ``nsteps`` steps (of the BDF1 scheme with ``bdf1``)."""
    st = initial_state(phi0, psi0, params, bdf1)
    for _ in range(nsteps):
        step(st, use_matrix)
    return st


# ---------------------------------------------------------------------------
# Physical free energy and arc length (Sec. 2.1)
# ---------------------------------------------------------------------------

def physical_energy(phi, psi, p: Params) -> Dict:
    """F = F^surf + F^bend + F^area + F^osm of eq. (energy_functional) with
    the densities of eq. (energy_densities), in the discrete forms of the
    scheme (cell |grad phi|^2, five-point Laplacian, h^2 sums); the arc
    length is int f_surf, the quantity F^area holds at A."""
    L = integral(f_surf(phi, p), p.h)
    omega = (phi ** 3 - phi) / p.eps - p.eps * lap(phi, p.h, p.bc)
    bend = p.gamma_bend * integral(3.0 * SQ2 / (16.0 * p.eps) * omega ** 2, p.h)
    surf = p.gamma_surf * L
    area = 0.5 * p.gamma_area * (L - p.A) ** 2
    pp = p_interp(phi)
    osm = integral(0.5 * (1.0 + pp) * f_in(psi, p) + 0.5 * (1.0 - pp) * f_out(psi, p), p.h)
    return dict(F=surf + bend + area + osm, surf=surf, bend=bend, area=area, osm=osm,
                arc_length=L)


# ---------------------------------------------------------------------------
# Smoothed initial conditions (App. F)
# ---------------------------------------------------------------------------

def smooth_ic(phi_sharp, h, eps, M=0.01, dt=1e-6, nsteps=10, use_matrix=None, clip=True):
    """Relax a sharp phase field by nsteps steps of the constant-mobility
    Cahn-Hilliard equation phi_t = M Lap((phi^3 - phi) / eps - eps Lap phi)
    with Neumann boundaries (App. F): first-order semi-implicit, the
    biharmonic term implicit and the nonlinear term explicit,
        (1/dt + M eps Lap_h^2) phi^{n+1} = phi^n / dt + (M / eps) Lap_h(phi^3 - phi)^n,
    solved with the DCT (App. C); then clip to [-1, 1]. App. F's choice is
    M = 0.01, dt = 1e-6 and T = 1e-5, i.e. ten steps. ``clip=False`` returns
    the field before clipping."""
    phi = np.array(phi_sharp, dtype=np.float64)
    ny, nx = phi.shape
    lam_h = neumann_lap_eigs(nx, ny, h)
    sigma = 1.0 / dt + M * eps * lam_h ** 2
    for _ in range(nsteps):
        rhs = phi / dt + (M / eps) * lap(phi ** 3 - phi, h)
        phi = spectral_solve(rhs, sigma, use_matrix)
    return np.clip(phi, -1.0, 1.0) if clip else phi


def ch_free_energy(phi, h, eps):
    """Free energy of the smoothing flow: int eps/2 |grad phi|^2 + (phi^2 - 1)^2 / (4 eps)."""
    gx = Dx(phi, h)
    gy = Dy(phi, h)
    grad = 0.5 * eps * (h * h * float(np.sum(gx * gx)) + h * h * float(np.sum(gy * gy)))
    return grad + integral((phi ** 2 - 1.0) ** 2 / (4.0 * eps), h)


# ---------------------------------------------------------------------------
# Energy and mass (Sec. 3.3, App. A, App. D)
# ---------------------------------------------------------------------------

def d_faces(psi_new, psis, phis, p: Params):
    """d^{n+1} = lambda D(psi^{n+1} - psi*) / sqrt(M_psi(A phi*)) on faces."""
    mx, my = face_mobility(phis, p)
    dpsi = psi_new - psis
    return (p.lam * Dx(dpsi, p.h, p.bc) / np.sqrt(mx),
            p.lam * Dy(dpsi, p.h, p.bc) / np.sqrt(my))


def d_norm_sq(psi_new, psis, phis, p: Params):
    """||d^{n+1}||^2 with the face inner products of App. D."""
    fx, fy = d_faces(psi_new, psis, phis, p)
    return face_ip(fx, fy, fx, fy, p.h)


def modified_energy(phi1, phi0, sav1, sav0, d_acc, p: Params) -> Dict:
    """E^{n+1,n}_mod of eq. (modified_discrete_energy) with discrete norms.

    ``phi1``/``sav1`` are level n+1, ``phi0``/``sav0`` level n, ``d_acc`` is
    sum_{j=2}^{n+1} (dt/2) ||d^j||^2.
    """
    h = p.h
    V1, U1, W1, Z1 = sav1
    V0, U0, W0, Z0 = sav0
    tt = theta_tilde(p)
    l1, l0 = lap(phi1, h, p.bc), lap(phi0, h, p.bc)
    bend = 0.5 * p.gamma_bend * 3.0 * SQ2 * p.eps / 8.0 * (
        ip(l1, l1, h) + ip(2.0 * l1 - l0, 2.0 * l1 - l0, h))
    g1 = grad_norm_sq(phi1, h, p.bc)
    g2 = grad_norm_sq(2.0 * phi1 - phi0, h, p.bc)
    gd = grad_norm_sq(phi1 - phi0, h, p.bc)
    surf = 0.5 * (p.gamma_surf * 3.0 * SQ2 * p.eps / 4.0 + p.theta) * (g1 + g2)
    stab = -0.5 * tt * (g1 + g2 - 2.0 * gd)
    lin = 0.5 * p.gamma_surf * 3.0 * SQ2 * p.beta / (4.0 * p.eps) * (
        ip(phi1, phi1, h) + ip(2.0 * phi1 - phi0, 2.0 * phi1 - phi0, h))
    sv = 0.5 * p.gamma_surf * 1.5 * SQ2 * (V1 ** 2 + (2.0 * V1 - V0) ** 2)
    su = 0.5 * p.gamma_area * (U1 ** 2 + (2.0 * U1 - U0) ** 2)
    sw = 0.5 * p.gamma_bend * 3.0 * SQ2 / (8.0 * p.eps) * (W1 ** 2 + (2.0 * W1 - W0) ** 2)
    sz = 0.5 * (Z1 ** 2 + (2.0 * Z1 - Z0) ** 2)
    parts = dict(bend=bend, surf=surf, stab=stab, lin=lin, V=sv, U=su, W=sw, Z=sz,
                 acc=-d_acc)
    parts["E"] = float(sum(parts.values()))
    return parts


def energy(st: State) -> Dict:
    """E^{n,n-1}_mod of the current state (levels n and n-1)."""
    if st.phi_prev is None:
        raise ValueError("energy needs two time levels")
    if st.bdf1:
        raise ValueError("E^{n,n-1}_mod is the energy of the BDF2 scheme")
    if st.scheme != "cc":
        raise ValueError("E^{n,n-1}_mod with the lambda-dissipation sum is the CC-MSAV energy")
    return modified_energy(st.phi, st.phi_prev, st.sav, st.sav_prev, st.d_acc, st.p)


def dissipation_terms(phi2, phi1, phi0, sav2, sav1, sav0, psi2, psis, phis, p: Params):
    """K^n and the right-hand side quantities of Thm. 3.1 for step n -> n+1.

    Level indices: 2 = n+1, 1 = n, 0 = n-1. Returns K^n, ||mu^{n+1}||^2 and
    ||c^{n+1} + d^{n+1}/2||^2, with mu^{n+1} from eq. (AC_BDF2) and
    nu^{n+1} = Z^{n+1} P* from eq. (nu_BDF2).
    """
    h = p.h
    tt = theta_tilde(p)
    sec = phi2 - 2.0 * phi1 + phi0
    lsec = lap(sec, h, p.bc)
    gsec = grad_norm_sq(sec, h, p.bc)
    Kn = (0.5 * p.gamma_bend * 3.0 * SQ2 * p.eps / 8.0 * ip(lsec, lsec, h)
          + 0.5 * (p.gamma_surf * 3.0 * SQ2 * p.eps / 4.0 + p.theta) * gsec
          + 1.5 * tt * gsec
          + 0.5 * p.gamma_surf * 3.0 * SQ2 * p.beta / (4.0 * p.eps) * ip(sec, sec, h))
    ssec = np.asarray(sav2) - 2.0 * np.asarray(sav1) + np.asarray(sav0)
    Kn += 0.5 * p.gamma_surf * 1.5 * SQ2 * ssec[0] ** 2
    Kn += 0.5 * p.gamma_area * ssec[1] ** 2
    Kn += 0.5 * p.gamma_bend * 3.0 * SQ2 / (8.0 * p.eps) * ssec[2] ** 2
    Kn += 0.5 * ssec[3] ** 2
    mu = -(3.0 * phi2 - 4.0 * phi1 + phi0) / (2.0 * p.dt * p.M_phi)
    mu_sq = ip(mu, mu, h)
    P = basis_P(phis, psis, p)
    nu = sav2[3] * P
    mx, my = face_mobility(phis, p)
    cx = np.sqrt(mx) * Dx(nu, h, p.bc)
    cy = np.sqrt(my) * Dy(nu, h, p.bc)
    dxf, dyf = d_faces(psi2, psis, phis, p)
    ex, ey = cx + 0.5 * dxf, cy + 0.5 * dyf
    cd_sq = face_ip(ex, ey, ex, ey, h)
    return Kn, mu_sq, cd_sq


def mass(st: State):
    """(h^2 sum psi, h^2 sum phi); only psi is conserved (App. D)."""
    return integral(st.psi, st.p.h), integral(st.phi, st.p.h)
