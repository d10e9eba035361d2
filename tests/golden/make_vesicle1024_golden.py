"""Write tests/golden/vesicle1024_oracle.npz: the FP64 oracle trajectory of the
N = 1024 perturbed-vesicle workload (seed 10057, 1000 steps).

Runs only the oracle (oracle/ccmsav_ref.py) on the seeded inputs of the
workload generator, five times: from the workload's initial fields (scipy's
FFT-based DCT, the oracle's default at this size); from the same fields with
the DCT written out as the cosine-matrix product (its definition: a different
rounding of every transform, as any other implementation has); from the
fields perturbed by one ulp with random signs (seeds 1 and 2); and with phi
and psi perturbed by one ulp with random signs after every step (seed 3).
At steps 1, 2, 250, 500 and 1000 it stores every eighth cell in each
direction of phi and psi of the first run, its SAVs at levels n and n-1, its
mass h^2 sum psi and modified energy, and the largest relative L-inf spread
(over the whole grid) of the other four runs from it: the rounding envelope
the GPU comparison is held to.

Usage (five oracle runs in parallel processes, about forty minutes):
    python tests/golden/make_vesicle1024_golden.py
"""
import os
import sys
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import ccmsav_ref as R  # noqa: E402
from workloads import make_workload  # noqa: E402

CHECKPOINTS = (1, 2, 250, 500, 1000)
STRIDE = 8


PER_STEP_SEED = 3
MATRIX_RUN = 4          # unperturbed, DCT as the cosine-matrix product


def trajectory(seed):
    from threadpoolctl import threadpool_limits
    # the matrix products use four threads, every other run one
    threadpool_limits(4 if seed == MATRIX_RUN else 1)
    use_matrix = seed == MATRIX_RUN
    m = make_workload("vesicle1024")[0]
    phi0, psi0 = m.phi0, m.psi0
    rng = np.random.default_rng(seed)
    ulp = 2.0 ** -52
    if seed in (1, 2):
        phi0 = phi0 * (1.0 + ulp * rng.choice([-1.0, 1.0], phi0.shape))
        psi0 = psi0 * (1.0 + ulp * rng.choice([-1.0, 1.0], psi0.shape))
    st = R.initial_state(phi0, psi0, m.params)
    out = {}
    for k in range(1, CHECKPOINTS[-1] + 1):
        R.step(st, use_matrix)
        if seed == PER_STEP_SEED:
            st.phi = st.phi * (1.0 + ulp * rng.choice([-1.0, 1.0], st.phi.shape))
            st.psi = st.psi * (1.0 + ulp * rng.choice([-1.0, 1.0], st.psi.shape))
        if k in CHECKPOINTS:
            out[k] = (st.phi.copy(), st.psi.copy(), st.sav.copy(), st.sav_prev.copy(),
                      R.mass(st)[0], R.energy(st)["E"])
        if k % 50 == 0:
            print(f"seed {seed}: step {k}", flush=True)
    return seed, out


def main():
    with Pool(5) as pool:
        runs = dict(pool.map(trajectory, (MATRIX_RUN, 0, 1, 2, PER_STEP_SEED)))
    rel = lambda a, b: float(np.abs(a - b).max() / np.abs(b).max())  # noqa: E731
    ref = runs[0]
    data = {}
    for k in CHECKPOINTS:
        phi, psi, sav, sav_prev, mass, energy = ref[k]
        env = [max(rel(o[k][0], phi), rel(o[k][1], psi), rel(o[k][2], sav))
               for o in (runs[1], runs[2], runs[PER_STEP_SEED], runs[MATRIX_RUN])]
        data[f"k{k}_phi"] = phi[::STRIDE, ::STRIDE]
        data[f"k{k}_psi"] = psi[::STRIDE, ::STRIDE]
        data[f"k{k}_sav"] = sav
        data[f"k{k}_sav_prev"] = sav_prev
        data[f"k{k}_mass"] = np.array(mass)
        data[f"k{k}_energy"] = np.array(energy)
        data[f"k{k}_env"] = np.array(env)
        print(f"step {k}: envelope {max(env):.2e} (ulp runs {max(env[:3]):.2e}, "
              f"matrix DCT {env[3]:.2e})", flush=True)
    np.savez_compressed(os.path.join(HERE, "vesicle1024_oracle.npz"), **data)


if __name__ == "__main__":
    main()
