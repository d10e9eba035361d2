"""Helpers shared by the parity tests: oracle trajectories and their rounding envelope.

The HIP path and the oracle round differently (summation order, FFT versus
matrix DCT), so after k steps they can only agree to within what the dynamics
make of ulp-level differences. That envelope is measured on the oracle alone:
the same run from inputs perturbed by one ulp (random sign per cell). A parity
bound at step k is max(1e-12, ENVELOPE_FACTOR * envelope_k).
"""
import numpy as np

from oracle import ccmsav_ref as R

BASE_TOL = 1e-12
ENVELOPE_FACTOR = 10.0


def rel_linf(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))


def oracle_trajectory(phi0, psi0, params, steps, perturb_seed=None, bdf1=False):
    """Oracle states after each of ``steps`` steps: list of (phi, psi, sav, sav_prev)
    (of the BDF1 scheme with ``bdf1``)."""
    if perturb_seed is not None:
        rng = np.random.default_rng(perturb_seed)
        ulp = 2.0 ** -52
        phi0 = phi0 * (1.0 + ulp * rng.choice([-1.0, 1.0], phi0.shape))
        psi0 = psi0 * (1.0 + ulp * rng.choice([-1.0, 1.0], psi0.shape))
    st = R.initial_state(phi0, psi0, params, bdf1)
    out = [(st.phi.copy(), st.psi.copy(), st.sav.copy(), st.sav.copy())]
    for _ in range(steps):
        R.step(st)
        out.append((st.phi, st.psi, st.sav.copy(), st.sav_prev.copy()))
    return out


def envelope(ref, pert):
    """Per-step max relative L-infinity difference of two oracle trajectories."""
    env = []
    for a, b in zip(ref, pert):
        env.append(max(rel_linf(a[0], b[0]), rel_linf(a[1], b[1]), rel_linf(a[2], b[2])))
    return env


def tolerances(env):
    return [max(BASE_TOL, ENVELOPE_FACTOR * e) for e in env]
