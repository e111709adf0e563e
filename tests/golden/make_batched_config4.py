"""Writes batched_config4.txt: oracle energies and adjoint gradients of the
first instance of each sector type in the batched workload.

Workload (config 4 of the benchmark set): synth.workload_batched(256, seed=0,
n_reps=2): instance i draws from default_rng([0, i]) its norb in {8, 10, 12},
n in {norb/2 - 1, norb/2}, LUCJ parameters N(0, 0.1) and a DF Hamiltonian with
L = norb terms.  For the first instance of each (norb, n) the oracle's energy
<psi|H|psi> and its adjoint gradient are stored.
Run: python tests/golden/make_batched_config4.py   (a few minutes on 8 cores)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import lucj as ol  # noqa: E402
from paper_2605_03123_amd import synth  # noqa: E402


def main():
    w = synth.workload_batched(256, seed=0, n_reps=2)
    first = {}
    for i, x in enumerate(w):
        first.setdefault((x.norb, x.nelec), i)
    t0 = time.time()
    with open(os.path.join(HERE, "batched_config4.txt"), "w") as f:
        f.write("# oracle energy and adjoint gradient, first instance of each sector type of\n")
        f.write("# synth.workload_batched(256, seed=0, n_reps=2); format: 'inst i norb n_a n_b energy'\n")
        f.write("# followed by one line of gradient entries\n")
        for (norb, nelec), i in sorted(first.items(), key=lambda kv: kv[1]):
            x = w[i]
            e, g = ol.grad_adjoint(x.data["params"], x.data["ham"], norb, nelec, x.data["n_reps"])
            f.write(f"inst {i} {norb} {nelec[0]} {nelec[1]} {float(np.real(e)):.17e}\n")
            f.write(" ".join(f"{v:.17e}" for v in g) + "\n")
        f.write(f"# written in {time.time() - t0:.0f} s\n")


if __name__ == "__main__":
    main()
