"""Pin for oracle/sampled.py: single amplitudes equal entries of the full compound-matrix rotation."""
import numpy as np

from oracle import gates as g
from oracle import sampled
from paper_2605_03123_amd import synth


def test_sampled_amplitudes_equal_full_rotation():
    r = synth.rng(31)
    norb, nelec = 7, (3, 4)
    vec = synth.random_state(r, 35, 35)
    Ua, Ub = synth.random_unitary(r, norb), synth.random_unitary(r, norb)
    full = g.apply_orbital_rotation(vec, Ua, norb, nelec, U_b=Ub)
    idx = [(0, 0), (3, 17), (34, 34), (20, 5)]
    out = sampled.rotated_amplitudes(vec, Ua, norb, nelec, idx, U_b=Ub)
    np.testing.assert_allclose(out, [full[i, j] for i, j in idx], atol=1e-14)
