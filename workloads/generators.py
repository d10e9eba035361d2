"""Seeded initial conditions and parameter sets for the vesicle workloads.

The paper's own initial conditions (an ellipse taken from earlier work, and
sharp polygonal shapes) are not specified numerically, so these synthetic
inputs stand in for them with the paper's parameter magnitudes:

* domain [0, L]^2 with L = 2*pi, N x N cell-centred grid, h = L / N,
  cell centres x_i = (i + 1/2) h (row-major arrays ``[ny][nx]``, x fastest);
* phase field phi0 = tanh((R(theta) - rho) / (sqrt(2) eps)) around the domain
  centre, R either a constant (circle) or 0.3 L (1 + sum_{m=2..8} a_m
  cos(m theta + theta_m)) with a_m ~ U(0, 0.05), theta_m ~ U(0, 2 pi);
* concentration psi0 = c_in (1 + phi0)/2 + c_out (1 - phi0)/2 (the affine
  form a phi0 + b used by the paper's growth/shrinkage tests), with the
  equilibrium concentrations psi_in = c_in - 0.35, psi_out = c_in + 0.35 so
  that c_out > c_in drives shrinkage and c_out < c_in growth;
* time step dt = 1e-4 for the circle; for the perturbed vesicles the paper's
  table value 1e-6 up to N = 1024, scaled by (1024 / N)^3 on finer grids;
  2.5e-8 for the members of the ensemble;
* the remaining coefficients from the paper's parameter table (App. G):
  gamma_surf = 1, gamma_bend = 1 (shrinkage) or 0.05 (growth),
  gamma_area = 5e4, gamma_in = gamma_out = 1e5, beta_in = beta_out = 0,
  M_phi = 1, M0 = 0.5, theta = 1.5, beta = 0, lambda = 1e5.

Random draws use ``numpy.random.default_rng(seed)`` in a fixed order per
member: a_2..a_8, then theta_2..theta_8, then c_out, then the eps choice.
Nothing here evaluates the scheme.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

DOMAIN_L = 2.0 * math.pi
# The circle case takes dt = 1e-4. The perturbed-vesicle family takes the
# paper's table value dt = 1e-6 up to N = 1024 and dt = 1e-6 (1024 / N)^3
# beyond: with eps = 4h the explicitly treated part of the bending term grows
# like 1/eps while the implicit fourth-order part shrinks like eps, so the
# step that keeps |phi| <= 1 scales like eps^3. Larger steps (1e-4 at N = 256,
# 1e-6 at N = 4096) drive phi* into the range where M_psi < 0 within a few
# steps, which the scheme's dissipation argument excludes.
DEFAULT_DT = 1.0e-4
VESICLE_DT = 1.0e-6
# The ensemble members (256^2 and 512^2, eps in {3h, 4h, 5h}) take 2.5e-8. At
# 1e-6 (and at 2.5e-7) these coarse members enter, after 10-100 steps, a regime
# in which the step amplifies per-step perturbations by several orders of
# magnitude within tens of steps, so no two roundings of the scheme agree
# there. At 1e-7 a third of the members still reach it between steps 500 and
# 2000: an FP64 run from inputs rounded to FP32 then ends 2e-4 - 6e-4 away.
# At 2.5e-8 (the same 2000 steps cover a quarter of that time) such runs stay
# within 3e-8 of the unrounded ones for every member over all 2000 steps.
ENSEMBLE_DT = 2.5e-8
PSI_GAP = 0.35


def vesicle_dt(n: int) -> float:
    """Time step of the perturbed-vesicle family on an n x n grid."""
    return VESICLE_DT * min(1.0, (1024.0 / n) ** 3)


def table_g_params(n: int, eps_cells: float, shrink: bool, c_in: float,
                   dt: float = DEFAULT_DT, length: float = DOMAIN_L) -> Dict:
    """Parameter set of the paper's table (App. G) on an n x n grid.

    ``eps_cells`` gives the interface width in cells (eps = eps_cells * h).
    ``A`` is NaN, meaning "use the discrete surface energy of phi0", which
    makes the arc-length SAV start at zero.
    """
    h = length / n
    return dict(
        nx=n, ny=n, h=h, dt=dt, eps=eps_cells * h,
        M_phi=1.0, M0=0.5,
        gamma_surf=1.0, gamma_bend=1.0 if shrink else 0.05, gamma_area=5.0e4,
        A=float("nan"),
        gamma_in=1.0e5, gamma_out=1.0e5,
        psi_in=c_in - PSI_GAP, psi_out=c_in + PSI_GAP,
        beta_in=0.0, beta_out=0.0,
        theta=1.5, lam=1.0e5, beta=0.0,
    )


# Parameter sets in which every coefficient differs from the App. G table, so
# that each term of the scheme carries its own weight: M_phi != 1 multiplies
# every Allen-Cahn constant, beta > 0 enters S~, r_S and C1, beta_in and
# beta_out differ and enter r_Z, gamma_in != gamma_out makes P~ asymmetric,
# and M0, theta, lambda all move. Row 0 is the reference set; the other rows
# vary it for the members of a mixed ensemble.
GENERAL_SETS = (
    dict(M_phi=0.7, M0=0.3, gamma_surf=1.3, gamma_bend=0.5, gamma_area=20.0,
         gamma_in=40.0, gamma_out=60.0, beta_in=0.2, beta_out=0.1,
         theta=3.0, lam=5.0, beta=0.3),
    dict(M_phi=1.4, M0=0.45, gamma_surf=0.8, gamma_bend=0.9, gamma_area=35.0,
         gamma_in=70.0, gamma_out=30.0, beta_in=0.05, beta_out=0.25,
         theta=1.0, lam=8.0, beta=0.15),
    dict(M_phi=0.5, M0=0.1, gamma_surf=1.6, gamma_bend=0.3, gamma_area=10.0,
         gamma_in=25.0, gamma_out=45.0, beta_in=0.3, beta_out=0.3,
         theta=4.5, lam=3.0, beta=0.5),
    dict(M_phi=1.1, M0=0.6, gamma_surf=1.15, gamma_bend=1.2, gamma_area=50.0,
         gamma_in=55.0, gamma_out=20.0, beta_in=0.15, beta_out=0.02,
         theta=2.0, lam=12.0, beta=0.05),
)


def general_dt(n: int) -> float:
    """Time step of the general parameter sets on a grid of n cells per side:
    1e-4 (16 / n)^2, where an FP64 run from inputs changed by one ulp stays
    within about 1e-13 of the unchanged run over 60 steps (16^2 .. 256^2)."""
    return 1.0e-4 * (16.0 / n) ** 2


def general_params(nx: int, ny: int, variant: int = 0, eps_cells: float = 4.0,
                   c_in: float = 1.0, dt: Optional[float] = None,
                   length: float = DOMAIN_L) -> Dict:
    """Parameters of GENERAL_SETS[variant] on an nx x ny grid with h = length / max(nx, ny)."""
    n = max(nx, ny)
    h = length / n
    p = dict(nx=nx, ny=ny, h=h, dt=general_dt(n) if dt is None else dt, eps=eps_cells * h,
             A=float("nan"), psi_in=c_in - PSI_GAP, psi_out=c_in + PSI_GAP)
    p.update(GENERAL_SETS[variant])
    return p


@dataclasses.dataclass
class Member:
    """One vesicle: initial fields plus its parameter dictionary."""
    name: str
    phi0: np.ndarray
    psi0: np.ndarray
    params: Dict
    meta: Dict


def _grid(n: int, length: float):
    h = length / n
    x = (np.arange(n, dtype=np.float64) + 0.5) * h
    X, Y = np.meshgrid(x, x, indexing="xy")   # X[j, i] = x_i, Y[j, i] = y_j
    return X - 0.5 * length, Y - 0.5 * length


def _fields(radius: np.ndarray, rho: np.ndarray, eps: float,
            c_in: float, c_out: float):
    phi0 = np.tanh((radius - rho) / (math.sqrt(2.0) * eps))
    psi0 = c_in * (1.0 + phi0) * 0.5 + c_out * (1.0 - phi0) * 0.5
    return np.ascontiguousarray(phi0), np.ascontiguousarray(psi0)


def circle_member(n: int, radius_frac: float = 0.25, eps_cells: float = 4.0,
                  c_in: float = 1.0, c_out: float = 1.2,
                  dt: float = DEFAULT_DT, length: float = DOMAIN_L,
                  name: Optional[str] = None) -> Member:
    """Centred circular vesicle of radius radius_frac * L."""
    X, Y = _grid(n, length)
    rho = np.hypot(X, Y)
    params = table_g_params(n, eps_cells, c_out > c_in, c_in, dt, length)
    phi0, psi0 = _fields(np.full_like(rho, radius_frac * length), rho,
                         params["eps"], c_in, c_out)
    return Member(name or f"circle{n}", phi0, psi0, params,
                  dict(c_in=c_in, c_out=c_out, radius_frac=radius_frac))


def vesicle_member(n: int, seed: int, c_out_range=(0.8, 1.2),
                   eps_choices=None, c_in: float = 1.0,
                   dt: Optional[float] = None, length: float = DOMAIN_L,
                   name: Optional[str] = None) -> Member:
    """Perturbed-circle vesicle R(theta) = 0.3 L (1 + sum a_m cos(m theta + theta_m))."""
    if dt is None:
        dt = vesicle_dt(n)
    rng = np.random.default_rng(seed)
    modes = np.arange(2, 9)
    amps = rng.uniform(0.0, 0.05, size=modes.size)
    phases = rng.uniform(0.0, 2.0 * math.pi, size=modes.size)
    c_out = float(rng.uniform(*c_out_range))
    if eps_choices is None:
        eps_cells = 4.0
    else:
        eps_cells = float(eps_choices[int(rng.integers(len(eps_choices)))])
    X, Y = _grid(n, length)
    rho = np.hypot(X, Y)
    ang = np.arctan2(Y, X)
    radius = 0.3 * length * (1.0 + sum(a * np.cos(m * ang + t)
                                       for m, a, t in zip(modes, amps, phases)))
    params = table_g_params(n, eps_cells, c_out > c_in, c_in, dt, length)
    phi0, psi0 = _fields(radius, rho, params["eps"], c_in, c_out)
    return Member(name or f"vesicle{n}_s{seed}", phi0, psi0, params,
                  dict(seed=seed, c_in=c_in, c_out=c_out, amps=amps.tolist(),
                       phases=phases.tolist(), eps_cells=eps_cells))


def general_member(nx: int, ny: int, seed: int, variant: int = 0,
                   eps_cells: float = 4.0) -> Member:
    """A perturbed vesicle (the recipe of vesicle_member on the square grid of
    max(nx, ny) cells, cut to ny x nx: the lower-left part for a rectangle)
    with the parameters of GENERAL_SETS[variant]."""
    n = max(nx, ny)
    base = vesicle_member(n, seed, eps_choices=None)
    params = general_params(nx, ny, variant, eps_cells)
    phi0 = np.ascontiguousarray(base.phi0[:ny, :nx])
    psi0 = np.ascontiguousarray(base.psi0[:ny, :nx])
    if eps_cells != 4.0:
        # re-profile the same boundary at this interface width
        phi0 = np.ascontiguousarray(np.tanh(np.arctanh(np.clip(phi0, -1 + 1e-15, 1 - 1e-15))
                                            * 4.0 / eps_cells))
        c_in, c_out = base.meta["c_in"], base.meta["c_out"]
        psi0 = np.ascontiguousarray(c_in * (1.0 + phi0) * 0.5 + c_out * (1.0 - phi0) * 0.5)
    return Member(f"general{nx}x{ny}_s{seed}_v{variant}", phi0, psi0, params,
                  dict(base.meta, variant=variant))


# Named workloads with their sizes and step counts.
WORKLOADS = {
    "circle128": dict(kind="single", n=128, steps=100),
    "vesicle1024": dict(kind="single", n=1024, steps=1000, seed=10057),
    "vesicle2048": dict(kind="single", n=2048, steps=500, seed=10057),
    "vesicle4096": dict(kind="single", n=4096, steps=500, seed=10057),
    "ensemble48x256_16x512": dict(kind="batch", steps=2000,
                                  members=[(256, 48), (512, 16)], seed0=10058,
                                  dt=ENSEMBLE_DT),
    "vesicle8192": dict(kind="single", n=8192, steps=200, seed=10057),
}


def make_workload(name: str, n_override: Optional[int] = None) -> List[Member]:
    """Materialise a named workload as a list of members.

    ``n_override`` shrinks a single-vesicle workload to another grid size with
    the same seed and recipe (used for small parity cases).
    """
    spec = WORKLOADS[name]
    if spec["kind"] == "single":
        n = n_override or spec["n"]
        if name.startswith("circle"):
            return [circle_member(n)]
        return [vesicle_member(n, spec["seed"])]
    members = []
    i = 0
    for n, count in spec["members"]:
        for _ in range(count):
            members.append(vesicle_member(
                n_override or n, spec["seed0"] + i, c_out_range=(0.8, 1.25),
                eps_choices=(3.0, 4.0, 5.0), dt=spec["dt"]))
            i += 1
    return members
