"""Write tests/golden/ensemble_member_oracle.npz: oracle trajectories of two
members of the 48 x 256^2 + 16 x 512^2 ensemble workload.

Runs only the FP64 oracle (oracle/ccmsav_ref.py) on the seeded inputs of the
workload generator: members 11 (N = 256, eps = 4h) and 17 (N = 256,
eps = 5h), 2000 steps each, three times: from the workload's initial
fields with the DCT written out as a matrix product (the definition), from
the same fields with scipy's FFT-based DCT instead (a different rounding of
every transform), and from the fields perturbed by one ulp with random signs
(seed 1). At steps 500, 1000 and 2000 it stores the SAVs and every fourth cell
in each direction of phi and psi of the first run, and the larger relative
L-inf spread (over the whole grid) of the other two runs from it: the
rounding envelope the GPU comparison is held to.

Usage (six oracle runs in parallel processes, about ten minutes):
    python tests/golden/make_ensemble_golden.py
"""
import os
import sys
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import ccmsav_ref as R  # noqa: E402
from workloads import make_workload  # noqa: E402

MEMBERS = (11, 17)
CHECKPOINTS = (500, 1000, 2000)


def trajectory(phi0, psi0, params, use_matrix=True):
    st = R.initial_state(phi0, psi0, params)
    out = {}
    for k in range(1, CHECKPOINTS[-1] + 1):
        R.step(st, use_matrix)
        if k in CHECKPOINTS:
            out[k] = (st.phi.copy(), st.psi.copy(), st.sav.copy())
    return out


def _run(job):
    i, kind = job
    m = make_workload("ensemble48x256_16x512")[i]
    phi0, psi0 = m.phi0, m.psi0
    if kind == "pert":
        rng = np.random.default_rng(1)
        ulp = 2.0 ** -52
        phi0 = phi0 * (1.0 + ulp * rng.choice([-1.0, 1.0], phi0.shape))
        psi0 = psi0 * (1.0 + ulp * rng.choice([-1.0, 1.0], psi0.shape))
    return job, trajectory(phi0, psi0, m.params, use_matrix=(kind != "alt"))


def main():
    jobs = [(i, kind) for i in MEMBERS for kind in ("ref", "alt", "pert")]
    with Pool(len(jobs)) as pool:
        runs = dict(pool.map(_run, jobs))
    rel = lambda a, b: float(np.abs(a - b).max() / np.abs(b).max())  # noqa: E731
    data = {}
    for i in MEMBERS:
        ref, alt, pert = runs[(i, "ref")], runs[(i, "alt")], runs[(i, "pert")]
        for k in CHECKPOINTS:
            phi, psi, sav = ref[k]
            env = [max(rel(o[k][0], phi), rel(o[k][1], psi), rel(o[k][2], sav))
                   for o in (alt, pert)]
            data[f"m{i}_k{k}_phi"] = phi[::4, ::4]
            data[f"m{i}_k{k}_psi"] = psi[::4, ::4]
            data[f"m{i}_k{k}_sav"] = sav
            data[f"m{i}_k{k}_env"] = np.array(env)
        print(f"member {i}: envelope " + ", ".join(
            f"{k}: {data[f'm{i}_k{k}_env'].max():.1e}" for k in CHECKPOINTS), flush=True)
    np.savez_compressed(os.path.join(HERE, "ensemble_member_oracle.npz"), **data)


if __name__ == "__main__":
    main()
