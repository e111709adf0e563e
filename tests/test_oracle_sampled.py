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


def test_blocked_amplitudes_equal_full_rotation():
    # row blocks smaller than the state, a complex64 state, and repeated columns
    r = synth.rng(32)
    norb, nelec = 8, (3, 4)
    vec = synth.random_state(r, 56, 70).astype(np.complex64)
    Ua, Ub = synth.random_unitary(r, norb), synth.random_unitary(r, norb)
    full = g.apply_orbital_rotation(vec.astype(np.complex128), Ua, norb, nelec, U_b=Ub)
    idx = [(0, 0), (3, 17), (55, 69), (20, 5), (41, 17)]
    out = sampled.rotated_amplitudes_blocked(vec, Ua, norb, nelec, idx, U_b=Ub, block=9)
    np.testing.assert_allclose(out, [full[i, j] for i, j in idx], atol=1e-14)
