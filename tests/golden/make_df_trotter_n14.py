"""Writes df_trotter_n14.txt: sampled amplitudes of two first-order DF Trotter
steps at norb = 14, (7, 7), computed by the oracle only.

Workload (config 2 of the benchmark set): DF Hamiltonian with L = 14 terms
from synth.workload_df_trotter(14, 14, seed=0) (h ~ sym N(0, 0.5), U_t real
orthogonal from QR, J_t ~ sym N(0, 0.1)), Hartree-Fock start, S_0 with
dt = 0.1, two steps (T = 0.2), one-body term applied first.  The oracle
applies every term without merging (compound matrices for each rotation).

Stored: the final norm, the energy <psi|H|psi>, and 4096 amplitudes at
indices drawn from default_rng([14, 7]) plus the first row's first 64 entries.
Run: python tests/golden/make_df_trotter_n14.py   (about 20 minutes on 8 cores)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import hamiltonian as oh  # noqa: E402
from paper_2605_03123_amd import synth  # noqa: E402

NORB, N, L, DT, STEPS = 14, 7, 14, 0.1, 2


def sample_indices(d):
    r = np.random.default_rng([14, 7])
    idx = np.stack([r.integers(0, d, 4096), r.integers(0, d, 4096)], axis=1)
    first = np.stack([np.zeros(64, dtype=np.int64), np.arange(64)], axis=1)
    return np.concatenate([first, idx])


def main():
    w = synth.workload_df_trotter(NORB, L, seed=0, start="hf", dt=DT, n_steps=STEPS)
    ham, vec = w.data["ham"], w.data["vec"]
    t0 = time.time()
    out = oh.simulate_trotter(vec, ham, DT * STEPS, NORB, (N, N), n_steps=STEPS, order=0)
    e = oh.df_energy(out, ham, NORB, (N, N))
    idx = sample_indices(out.shape[0])
    with open(os.path.join(HERE, "df_trotter_n14.txt"), "w") as f:
        f.write("# oracle: two S_0 steps, dt = 0.1, norb = 14 (7,7), L = 14, seed 0, HF start\n")
        f.write(f"# written by tests/golden/make_df_trotter_n14.py in {time.time() - t0:.0f} s\n")
        f.write(f"norm {np.linalg.norm(out):.17e}\n")
        f.write(f"energy {e.real:.17e} {e.imag:.17e}\n")
        for i, j in idx:
            a = out[i, j]
            f.write(f"{i} {j} {a.real:.17e} {a.imag:.17e}\n")


if __name__ == "__main__":
    main()
