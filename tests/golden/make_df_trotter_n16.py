"""Writes df_trotter_n16.txt: sampled amplitudes, norm and energy of one
first-order DF Trotter step at norb = 16, (8, 8), computed by the oracle only.

Workload (the benchmark's DF step): DF Hamiltonian with L = 16 terms from
synth.workload_df_trotter(16, 16, seed=0, start="random") (h ~ sym N(0, 0.5),
U_t real orthogonal from QR, J_t ~ sym N(0, 0.1)), then the seed-0 random
normalized start state; S_0 with dt = 0.1, one step, one-body term applied
first.  The oracle applies every term without merging: 33 orbital rotations
as compound-matrix products and 16 diagonal-Coulomb phases.

A second oracle run starts from the same state rounded to complex64 and
upcast (the input a complex64 run sees), so that the complex64 error can be
stated both against the original input and against the rounded one.

Stored: the wall time of each oracle step and the host cores it used; the
final norm; the energy <psi|H|psi> of the first run; 4096 amplitudes at
indices drawn from default_rng([16, 8]) plus the first row's first 64
entries, from both runs.
Run: python tests/golden/make_df_trotter_n16.py   (about 2 hours on 8 cores, ~20 GB)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import gates as og  # noqa: E402
from oracle import hamiltonian as oh  # noqa: E402
from paper_2605_03123_amd import synth  # noqa: E402

NORB, N, L, DT = 16, 8, 16, 0.1


def sample_indices(d):
    r = np.random.default_rng([16, 8])
    idx = np.stack([r.integers(0, d, 4096), r.integers(0, d, 4096)], axis=1)
    first = np.stack([np.zeros(64, dtype=np.int64), np.arange(64)], axis=1)
    return np.concatenate([first, idx])


def main():
    cores = len(os.sched_getaffinity(0))
    og.set_workers(cores)
    w = synth.workload_df_trotter(NORB, L, seed=0, start="random", dt=DT)
    ham, vec = w.data["ham"], w.data["vec"]
    idx = sample_indices(vec.shape[0])

    t0 = time.time()
    out = oh.simulate_trotter(vec, ham, DT, NORB, (N, N), n_steps=1, order=0)
    t_step = time.time() - t0
    print(f"step (original input): {t_step:.0f} s", flush=True)
    t0 = time.time()
    e = oh.df_energy(out, ham, NORB, (N, N))
    t_energy = time.time() - t0
    print(f"energy: {t_energy:.0f} s", flush=True)
    amps = out[idx[:, 0], idx[:, 1]].copy()
    norm = np.linalg.norm(out)
    del out

    vec64 = vec.astype(np.complex64).astype(np.complex128)
    del vec
    t0 = time.time()
    out64 = oh.simulate_trotter(vec64, ham, DT, NORB, (N, N), n_steps=1, order=0)
    t_step64 = time.time() - t0
    print(f"step (complex64-rounded input): {t_step64:.0f} s", flush=True)
    amps64 = out64[idx[:, 0], idx[:, 1]].copy()
    norm64 = np.linalg.norm(out64)
    del out64

    with open(os.path.join(HERE, "df_trotter_n16.txt"), "w") as f:
        f.write("# oracle: one S_0 step, dt = 0.1, norb = 16 (8,8), L = 16, seed 0, random start\n")
        f.write("# written by tests/golden/make_df_trotter_n16.py\n")
        f.write(f"# oracle step wall time {t_step:.1f} s (rounded input {t_step64:.1f} s), energy {t_energy:.1f} s,"
                f" {cores} host cores\n")
        f.write(f"step_seconds {t_step:.3f} {cores}\n")
        f.write(f"norm {norm:.17e}\n")
        f.write(f"norm_c64_input {norm64:.17e}\n")
        f.write(f"energy {e.real:.17e} {e.imag:.17e}\n")
        f.write("# i j re im re_c64_input im_c64_input\n")
        for (i, j), a, b in zip(idx, amps, amps64):
            f.write(f"{i} {j} {a.real:.17e} {a.imag:.17e} {b.real:.17e} {b.imag:.17e}\n")


if __name__ == "__main__":
    main()
