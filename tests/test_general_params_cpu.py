"""The general parameter sets of the GPU parity tests expose every term.

With the App. G parameters (M_phi = 1, beta = beta_in = beta_out = 0,
gamma_in = gamma_out) a dropped M_phi factor, a wrong sign of beta, a dropped
beta_in/beta_out or a swap of gamma_in and gamma_out leaves the step
unchanged. Each test below plants one such slip in the oracle (on the CPU)
and checks that, on general_member's inputs, eight steps move by far more
than the GPU parity bound of 1e-12 (the rounding envelope of these runs is
about 1e-14). A step that carries the slip therefore cannot pass the GPU
parity tests of tests/test_gpu_params.py.
"""
import dataclasses

import numpy as np
import pytest

from oracle import ccmsav_ref as R
from workloads import GENERAL_SETS, general_member

STEPS = 8
# far above the GPU bar: a slip must move the result by at least this much
DETECT = 1e-8


def run(m, steps=STEPS, bdf1=False):
    st = R.initial_state(m.phi0, m.psi0, m.params, bdf1)
    for _ in range(steps):
        R.step(st)
    return st


def moved(a, b):
    return max(np.abs(a.phi - b.phi).max() / np.abs(b.phi).max(),
               np.abs(a.psi - b.psi).max() / np.abs(b.psi).max(),
               np.abs(a.sav - b.sav).max() / np.abs(b.sav).max())


@pytest.fixture(scope="module")
def member():
    return general_member(16, 16, 10057)


@pytest.fixture(scope="module")
def clean(member):
    return run(member)


def _orig(name):
    return getattr(R, name)


SLIPS = {
    # the M_phi factor of the theta~ Laplacian term of f (eq. AC_BDF2)
    "theta_term_without_M_phi": ("theta_tilde", lambda f: lambda p: f(p) / p.M_phi),
    # M_phi missing from C2 or C3 of chi (App. B, Step 3)
    "C2_without_M_phi": ("chi_coefficients",
                         lambda f: lambda p, a: (f(p, a)[0], f(p, a)[1] / p.M_phi, f(p, a)[2])),
    "C3_without_M_phi": ("chi_coefficients",
                         lambda f: lambda p, a: (f(p, a)[0], f(p, a)[1], f(p, a)[2] / p.M_phi)),
    # M_phi missing from the beta part of C1
    "C1_beta_part_without_M_phi": ("chi_coefficients",
                                   lambda f: lambda p, a: ((f(p, a)[0] - a) / p.M_phi + a,
                                                           f(p, a)[1], f(p, a)[2])),
    # M_phi missing from one SAV weight c_gs / c_go
    "c_gs_without_M_phi": ("sav_weights",
                           lambda f: lambda p: (f(p)[0] / p.M_phi,) + tuple(f(p)[1:])),
    "c_go_without_M_phi": ("sav_weights",
                           lambda f: lambda p: tuple(f(p)[:3]) + (f(p)[3] / p.M_phi,)),
    # wrong sign of beta in S~ and its normaliser r_S
    "beta_sign_in_S": ("basis_S",
                       lambda f: lambda phi, p: f(phi, dataclasses.replace(p, beta=-p.beta))),
    # beta_in, beta_out dropped from the osmotic energies (r_Z, K~)
    "beta_in_dropped": ("f_in", lambda f: lambda psi, p: f(psi, p) - p.beta_in),
    "beta_out_dropped": ("f_out", lambda f: lambda psi, p: f(psi, p) - p.beta_out),
    # gamma_in and gamma_out swapped in P~
    "gammas_swapped_in_P": ("basis_P",
                            lambda f: lambda phi, psi, p: f(phi, psi, dataclasses.replace(
                                p, gamma_in=p.gamma_out, gamma_out=p.gamma_in))),
    # mobility with the App. G value M0 = 0.5 instead of the parameter
    "M0_fixed": ("mobility_psi",
                 lambda f: lambda phi, p: f(phi, dataclasses.replace(p, M0=0.5))),
}


@pytest.mark.parametrize("slip", sorted(SLIPS))
def test_planted_slip_moves_the_step(member, clean, monkeypatch, slip):
    name, wrap = SLIPS[slip]
    monkeypatch.setattr(R, name, wrap(_orig(name)))
    got = run(member)
    assert moved(got, clean) > DETECT, slip


def test_general_sets_differ_from_table_g_in_every_coefficient():
    table_g = dict(M_phi=1.0, M0=0.5, gamma_surf=1.0, gamma_in=1e5, gamma_out=1e5,
                   beta_in=0.0, beta_out=0.0, theta=1.5, lam=1e5, beta=0.0)
    for s in GENERAL_SETS:
        for k, v in table_g.items():
            assert s[k] != v, k
        assert s["gamma_in"] != s["gamma_out"] or s["beta_in"] != s["beta_out"]
        assert s["beta"] > 0.0 and s["M_phi"] != 1.0


def test_general_member_rounding_envelope_is_small(member):
    """One-ulp input changes stay near 1e-14 over the eight steps, so the
    GPU comparison at max(1e-12, 10 x envelope) is the 1e-12 bar."""
    rng = np.random.default_rng(1)
    ulp = 2.0 ** -52
    pert = dataclasses.replace(member)
    pert.phi0 = member.phi0 * (1.0 + ulp * rng.choice([-1.0, 1.0], member.phi0.shape))
    pert.psi0 = member.psi0 * (1.0 + ulp * rng.choice([-1.0, 1.0], member.psi0.shape))
    assert moved(run(pert), run(member)) < 1e-13
